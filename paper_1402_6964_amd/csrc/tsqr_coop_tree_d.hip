// Cooperative FP64 tree launches for 25..32 columns.
#include "tsqr_coop_tree.hpp"

namespace tsnmf {

hipError_t launch_coop_tree_25_32(int n, const TreeArgs& t, hipStream_t stream) {
    switch (n) {
        case 25: return launch_coop_tree_n<25>(t, stream);
        case 26: return launch_coop_tree_n<26>(t, stream);
        case 27: return launch_coop_tree_n<27>(t, stream);
        case 28: return launch_coop_tree_n<28>(t, stream);
        case 29: return launch_coop_tree_n<29>(t, stream);
        case 30: return launch_coop_tree_n<30>(t, stream);
        case 31: return launch_coop_tree_n<31>(t, stream);
        case 32: return launch_coop_tree_n<32>(t, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tsnmf
