// Cooperative FP64 leaf launches for 1..16 columns (row-major input).
#include "tsqr_coop_leaf.hpp"

namespace tsnmf {

hipError_t launch_coop_leaf_1_16(int n, const StreamArgs& a, hipStream_t stream) {
    switch (n) {
        case 1: return launch_coop_leaf_n<1>(a, stream);
        case 2: return launch_coop_leaf_n<2>(a, stream);
        case 3: return launch_coop_leaf_n<3>(a, stream);
        case 4: return launch_coop_leaf_n<4>(a, stream);
        case 5: return launch_coop_leaf_n<5>(a, stream);
        case 6: return launch_coop_leaf_n<6>(a, stream);
        case 7: return launch_coop_leaf_n<7>(a, stream);
        case 8: return launch_coop_leaf_n<8>(a, stream);
        case 9: return launch_coop_leaf_n<9>(a, stream);
        case 10: return launch_coop_leaf_n<10>(a, stream);
        case 11: return launch_coop_leaf_n<11>(a, stream);
        case 12: return launch_coop_leaf_n<12>(a, stream);
        case 13: return launch_coop_leaf_n<13>(a, stream);
        case 14: return launch_coop_leaf_n<14>(a, stream);
        case 15: return launch_coop_leaf_n<15>(a, stream);
        case 16: return launch_coop_leaf_n<16>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

// Short FP64 slabs, 1 <= n <= 32 (row-major, any row stride).
hipError_t launch_coop_leaf_f64(int n, const StreamArgs& a, hipStream_t stream) {
    return n <= 16 ? launch_coop_leaf_1_16(n, a, stream) : launch_coop_leaf_17_32(n, a, stream);
}

}  // namespace tsnmf
