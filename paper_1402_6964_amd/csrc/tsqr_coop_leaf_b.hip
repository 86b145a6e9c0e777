// Cooperative FP64 leaf launches for 17..32 columns (row-major input).
#include "tsqr_coop_leaf.hpp"

namespace tsnmf {

hipError_t launch_coop_leaf_17_32(int n, const StreamArgs& a, hipStream_t stream) {
    switch (n) {
        case 17: return launch_coop_leaf_n<17>(a, stream);
        case 18: return launch_coop_leaf_n<18>(a, stream);
        case 19: return launch_coop_leaf_n<19>(a, stream);
        case 20: return launch_coop_leaf_n<20>(a, stream);
        case 21: return launch_coop_leaf_n<21>(a, stream);
        case 22: return launch_coop_leaf_n<22>(a, stream);
        case 23: return launch_coop_leaf_n<23>(a, stream);
        case 24: return launch_coop_leaf_n<24>(a, stream);
        case 25: return launch_coop_leaf_n<25>(a, stream);
        case 26: return launch_coop_leaf_n<26>(a, stream);
        case 27: return launch_coop_leaf_n<27>(a, stream);
        case 28: return launch_coop_leaf_n<28>(a, stream);
        case 29: return launch_coop_leaf_n<29>(a, stream);
        case 30: return launch_coop_leaf_n<30>(a, stream);
        case 31: return launch_coop_leaf_n<31>(a, stream);
        case 32: return launch_coop_leaf_n<32>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tsnmf
