// Layer kernels with 8-bit float message storage.
#include "layer.h"

hipError_t qm_layer_f8(const LayerArgs &a, int mode, int maxd, int fpl, int block, int hint, hipStream_t s) {
    return layer_msg<Fp8Msg>(a, mode, maxd, fpl, block, hint, s);
}

hipError_t qm_layer_multi_f8(const MultiLayerArgs &m, int maxd, int fpl, int block, int hint, hipStream_t s) {
    return layer_multi_msg<Fp8Msg>(m, maxd, fpl, block, hint, s);
}
