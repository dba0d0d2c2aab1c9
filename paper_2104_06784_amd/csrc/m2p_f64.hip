// FP64 kernels: compiled without FMA contraction so that the arithmetic is
// evaluated exactly as written (bitwise reproducible against plain C).
#define M2P_REAL double
#include "m2p_kernels_impl.h"
