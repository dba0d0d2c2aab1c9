// m2p_host.h -- host helpers shared by the single-scenario and the batched
// C ABI implementations.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "m2p.h"
#include "m2p_device.h"

namespace m2p {

int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
size_t round_up(size_t a, size_t m);
int validate_scenario(const m2p_grid* g, const m2p_params* p, int32_t prec, const double* dem);
KParams make_kparams(const m2p_grid* g, const m2p_params* p, bool has_mu);
std::vector<double> padded_dem(const KParams& K, const double* dem, double L);
int outflow_volumes(const double* bpart_dev, int nmax, int nx, int ny, const KParams& K, hipStream_t st,
                    double* out_s, double* out_f);

}  // namespace m2p

#define HIPCHK(x)                                      \
    do {                                               \
        hipError_t e_ = (x);                           \
        if (e_ != hipSuccess) return m2p::hip_fail(e_, #x); \
    } while (0)
