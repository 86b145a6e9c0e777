// Cooperative FP64 tree launches for 17..24 columns.
#include "tsqr_coop_tree.hpp"

namespace tsnmf {

hipError_t launch_coop_tree_17_24(int n, const TreeArgs& t, hipStream_t stream) {
    switch (n) {
        case 17: return launch_coop_tree_n<17>(t, stream);
        case 18: return launch_coop_tree_n<18>(t, stream);
        case 19: return launch_coop_tree_n<19>(t, stream);
        case 20: return launch_coop_tree_n<20>(t, stream);
        case 21: return launch_coop_tree_n<21>(t, stream);
        case 22: return launch_coop_tree_n<22>(t, stream);
        case 23: return launch_coop_tree_n<23>(t, stream);
        case 24: return launch_coop_tree_n<24>(t, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tsnmf
