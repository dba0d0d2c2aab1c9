// m2p_launch.h -- host-side launch interface between the C ABI and the
// per-precision kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "m2p_device.h"

namespace m2p {

struct Bufs {
    void* U;             // state U^n (6 fields, [ny][pitch] each)
    void* Us;            // stage state U*
    const void* b;       // padded DEM / L
    const void* mu;      // per-cell tan(delta_b) or nullptr
    DevScalars* S;       // device scalars
    double* bpart;       // boundary outflow partials [2][4][nmax][2]
    const double* tables;  // inflow hydrographs
    double* mass_part;   // [2 * kMassBlocks]
    int nbx, nby, nmax;  // stage-kernel grid and partial stride
};

constexpr int kMassBlocks = 1024;

template <typename T>
struct Launch {
    // part 0: stage 1, part 1: stage 2, part 2: finalize
    static hipError_t step_part(const KParams& P, const Bufs& B, hipStream_t st, int variant, int rows, int part);
    static hipError_t init(const KParams& P, const Bufs& B, hipStream_t st);
    static hipError_t set_state(const KParams& P, const Bufs& B, const double* f, int vertical, int has_v,
                                hipStream_t st);
    static hipError_t get_fields(const KParams& P, const Bufs& B, double* f, hipStream_t st);
    static hipError_t mass(const KParams& P, const Bufs& B, hipStream_t st);
    static void grid_dims(const KParams& P, int variant, int rows, int& nbx, int& nby);
};

}  // namespace m2p
