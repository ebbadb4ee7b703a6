// Layer kernels with float32 message storage.
#include "layer.h"

hipError_t qm_layer_f32(const LayerArgs &a, int mode, int maxd, int fpl, int block, int hint, hipStream_t s) {
    return layer_msg<float>(a, mode, maxd, fpl, block, hint, s);
}

hipError_t qm_layer_multi_f32(const MultiLayerArgs &m, int maxd, int fpl, int block, int hint, hipStream_t s) {
    return layer_multi_msg<float>(m, maxd, fpl, block, hint, s);
}
