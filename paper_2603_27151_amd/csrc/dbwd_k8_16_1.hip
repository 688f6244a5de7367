// Backward fragment decode instantiated for the MLP shape (8, 16, 1).
#include "decode_bwd_impl.hpp"

namespace soup {

void launch_decode_bwd_k8_16_1(const DecodeArgs& a, bool logp, hipStream_t s) {
    launch_decode_bwd_s<MlpShape<8, 16, 1>>(a, logp, s);
}

size_t decode_bwd_lds_k8_16_1(int G, bool logp) { return decode_bwd_lds_s<MlpShape<8, 16, 1>>(G, logp); }

void launch_fragment_gates_k8_16_1(const DecodeArgs& a, uint32_t* gates_out, hipStream_t s) {
    launch_fragment_gates_s<MlpShape<8, 16, 1>>(a, gates_out, s);
}

}  // namespace soup
