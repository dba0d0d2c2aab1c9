// m2p_launch.h -- host-side launch interface between the C ABI and the
// per-precision kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "m2p_device.h"

namespace m2p {

// Launch shape of the stage kernels for one variant.
struct Shape {
    int variant;       // 1 reference, 2 tiled
    int nbx, nby;      // reference: 64 x 4 blocks
    int R, nstrips, nrb;  // tiled: rows per wavefront, strips, row blocks
    int n_we, n_sn;    // boundary partials per W/E and per S/N side
    int nw;            // per-stage partial slots
    int blocks;        // workgroups per stage launch
    int global_addr;   // tiled: 64-bit global addresses even where raw buffer offsets would reach
};

struct Bufs {
    void* U;               // state U^n (6 fields, [ny][pitch] each)
    void* Us;              // stage state U*
    void* Us2;             // second stage state of the three-stage method (else nullptr)
    void* Uout;            // output of the step's last stage (nullptr: in place over U)
    void* kep;             // earth-pressure coefficients [2][ny][pitch] (the option only, else nullptr)
    const void* b;         // padded DEM / L
    const void* mu;        // per-cell tan(delta_b) or nullptr
    DevScalars* S;         // device scalars
    double* bpart;         // outflow integrals and stage values per boundary face [kOutSlots][4][nmax][2]
    double* wpart;         // per-wave / per-block partials [stages][nw][4]
    const double* tables;  // inflow hydrographs
    double* mass_part;     // [2 * kMassBlocks]
    int nmax;              // stride of bpart
    int nw_ref;            // partial slots of the reference grid (speeds kernel)
};

constexpr int kMassBlocks = 1024;

// Finalize: one workgroup of kFinThreads per scenario.
constexpr int kFinThreads = 256;
constexpr int kFinVals = 4;  // 2 speed maxima, clamps, non-finite flag
constexpr int kOutSlots = 4;  // outflow integrals + the values of up to three stages
// index of the step's dt in bpart, after the slots (the buffer holds 2 more doubles)
constexpr size_t outflow_dt_index(int nmax) { return (size_t)kOutSlots * 4 * nmax * 2; }

// Scenario record of a batched ensemble: constants and device pointers.
template <typename T>
struct ScenDesc {
    KParams P;
    T* U;
    T* Us;
    const T* b;
    const T* mu;
    DevScalars* S;
    double* bpart;
    double* wpart;
    const double* tables;
    int nmax, nstrips, nrb, nw_ref;
};

Shape make_shape(const KParams& P, int variant, int rows, int slots);

template <typename T>
struct Launch {
    // parts 0 .. P.rk - 1: the stages of a step, part P.rk: finalize
    static hipError_t step_part(const KParams& P, const Bufs& B, const Shape& sh, hipStream_t st, int part);
    static hipError_t init(const KParams& P, const Bufs& B, hipStream_t st);
    // wavefronts of the tiled stage-2 kernel the current device holds at
    // once (its occupancy times the compute units), 0 if unknown
    static int resident_waves(const KParams& P);
    static hipError_t set_state(const KParams& P, const Bufs& B, const double* f, int vertical, int has_v,
                                hipStream_t st);
    static hipError_t get_fields(const KParams& P, const Bufs& B, double* f, hipStream_t st);
    static hipError_t mass(const KParams& P, const Bufs& B, hipStream_t st);
    // batched ensemble: part 0 / 1 = persistent stage kernels over the work
    // list, part 2 = one finalize workgroup per scenario (mode 0 or 1)
    static hipError_t batch_part(const ScenDesc<T>* scen, int nscen, const int* work, int nwork, int R, int blocks,
                                 bool buf,
                                 hipStream_t st, int part, int mode);
    // adjoint support (buffers are [6][ny][pitch] state-shaped unless noted)
    static hipError_t jvp(const KParams& P, const Bufs& B, const void* U, const void* dU, const void* dmu, int stage,
                          void* E, void* dE, hipStream_t st);
    // lam_in = transpose of the stage applied to lscale * lam, plus zc * z if z
    // is given (z may alias lam_in)
    static hipError_t vjp(const KParams& P, const Bufs& B, const void* U, const void* lam, double lscale,
                          int stage, double dt, void* GT, void* DU, void* FCX, void* FCY, void* SC, void* lam_in,
                          const void* z, double zc, void* gmu, hipStream_t st);
    static hipError_t loss(const KParams& P, const Bufs& B, const void* U, const double* target, void* lam,
                           double* part, hipStream_t st);
    static hipError_t dot(const KParams& P, const void* x, const void* y, double* part, hipStream_t st);
};

}  // namespace m2p
