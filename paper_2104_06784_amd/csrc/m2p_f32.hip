// FP32-state kernels: FP32 arithmetic with fused multiply-adds and fast
// reciprocal / square root; time, dt and volume sums stay FP64.
#define M2P_REAL float
#include "m2p_kernels_impl.h"
