// Layer kernels with IEEE binary16 message storage.
#include "layer.h"

hipError_t qm_layer_f16(const LayerArgs &a, int mode, int maxd, int fpl, int block, int hint, hipStream_t s) {
    return layer_msg<_Float16>(a, mode, maxd, fpl, block, hint, s);
}

hipError_t qm_layer_multi_f16(const MultiLayerArgs &m, int maxd, int fpl, int block, int hint, hipStream_t s) {
    return layer_multi_msg<_Float16>(m, maxd, fpl, block, hint, s);
}
