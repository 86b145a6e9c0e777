// Cooperative FP64 tree launches for 9..16 columns.
#include "tsqr_coop_tree.hpp"

namespace tsnmf {

hipError_t launch_coop_tree_9_16(int n, const TreeArgs& t, hipStream_t stream) {
    switch (n) {
        case 9: return launch_coop_tree_n<9>(t, stream);
        case 10: return launch_coop_tree_n<10>(t, stream);
        case 11: return launch_coop_tree_n<11>(t, stream);
        case 12: return launch_coop_tree_n<12>(t, stream);
        case 13: return launch_coop_tree_n<13>(t, stream);
        case 14: return launch_coop_tree_n<14>(t, stream);
        case 15: return launch_coop_tree_n<15>(t, stream);
        case 16: return launch_coop_tree_n<16>(t, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tsnmf
