// Per-message-type layer launchers (layer_f32.hip, layer_f16.hip,
// layer_f8.hip).  mode: 0 layered sweep, 1 early-terminating sweep,
// 2 check half of a flooding iteration.
#pragma once

#include "qcmet_internal.h"

hipError_t qm_layer_f32(const LayerArgs &a, int mode, int maxd, int fpl, int block, int hint, hipStream_t s);
hipError_t qm_layer_f16(const LayerArgs &a, int mode, int maxd, int fpl, int block, int hint, hipStream_t s);
hipError_t qm_layer_f8(const LayerArgs &a, int mode, int maxd, int fpl, int block, int hint, hipStream_t s);
hipError_t qm_layer_multi_f32(const MultiLayerArgs &m, int maxd, int fpl, int block, int hint, hipStream_t s);
hipError_t qm_layer_multi_f16(const MultiLayerArgs &m, int maxd, int fpl, int block, int hint, hipStream_t s);
hipError_t qm_layer_multi_f8(const MultiLayerArgs &m, int maxd, int fpl, int block, int hint, hipStream_t s);
