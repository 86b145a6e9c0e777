// Cooperative FP64 tree launches for 1..8 columns.
#include "tsqr_coop_tree.hpp"

namespace tsnmf {

hipError_t launch_coop_tree_1_8(int n, const TreeArgs& t, hipStream_t stream) {
    switch (n) {
        case 1: return launch_coop_tree_n<1>(t, stream);
        case 2: return launch_coop_tree_n<2>(t, stream);
        case 3: return launch_coop_tree_n<3>(t, stream);
        case 4: return launch_coop_tree_n<4>(t, stream);
        case 5: return launch_coop_tree_n<5>(t, stream);
        case 6: return launch_coop_tree_n<6>(t, stream);
        case 7: return launch_coop_tree_n<7>(t, stream);
        case 8: return launch_coop_tree_n<8>(t, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_coop_tree(int n, const TreeArgs& t, hipStream_t stream) {
    if (n <= 8) return launch_coop_tree_1_8(n, t, stream);
    if (n <= 16) return launch_coop_tree_9_16(n, t, stream);
    if (n <= 24) return launch_coop_tree_17_24(n, t, stream);
    return launch_coop_tree_25_32(n, t, stream);
}

}  // namespace tsnmf
