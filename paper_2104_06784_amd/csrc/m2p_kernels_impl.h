// m2p_kernels_impl.h -- launchers for one precision (included by
// m2p_f64.hip / m2p_f32.hip after defining M2P_REAL).
#pragma once

#include "m2p_kernels.h"
#include "m2p_tiled.h"
#include "m2p_adjoint.h"

namespace m2p {

template <>
hipError_t Launch<M2P_REAL>::step_part(const KParams& P, const Bufs& B, const Shape& sh, hipStream_t st, int part)
{
    using T = M2P_REAL;
    T* U = (T*)B.U;
    T* Us = (T*)B.Us;
    T* Us2 = (T*)B.Us2;
    const T* b = (const T*)B.b;
    const T* mu = (const T*)B.mu;
    if (part == P.rk) {
        // small grids: one wavefront (shorter combining passes)
        if (sh.nw <= 512)
            hipLaunchKernelGGL((k_finalize<T, 64>), dim3(1 + (4 * B.nmax + 63) / 64), dim3(64), 0, st, P, B.S,
                               B.tables, 0, B.wpart, sh.nw, B.bpart, B.nmax);
        else
            hipLaunchKernelGGL((k_finalize<T>), dim3(1 + (4 * B.nmax + kFinThreads - 1) / kFinThreads),
                               dim3(kFinThreads), 0, st, P, B.S, B.tables, 0, B.wpart, sh.nw, B.bpart, B.nmax);
        return hipGetLastError();
    }
    // Heun: E(U) -> Us, then (U + E(Us)) / 2 -> U.  Three-stage: E(U) -> Us,
    // 3/4 U + 1/4 E(Us) -> Us2, then 1/3 U + 2/3 E(Us2) -> U.
    const int kind = part == 0 ? 1 : (P.rk == 2 ? 2 : (part == 1 ? 3 : 4));
    const T* in = part == 0 ? U : (kind == 4 ? Us2 : Us);
    T* out = part == 0 ? Us : (kind == 3 ? Us2 : (B.Uout ? (T*)B.Uout : U));
    if ((P.flags & kFlagEarthPressure) && sh.variant == 1) {
        // the option's coefficients of the stage input for the reference
        // kernel (the tiled kernel computes them in its march)
        if (!B.kep) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_earth_pressure<T>), dim3(sh.nbx, sh.nby), dim3(64, 4), 0, st, P, in, b, mu,
                           (T*)B.kep);
    }
    if (sh.variant == 1) {
        dim3 blk(64, 4), grd(sh.nbx, sh.nby);
#define M2P_REF(K)                                                                                              \
    do {                                                                                                        \
        if (P.flags & kFlagWellBalanced)                                                                        \
            hipLaunchKernelGGL((k_stage_ref<T, K, true>), grd, blk, 0, st, P, in, U, out, b, mu, B.S, B.bpart,  \
                               B.wpart, B.nmax, (const T*)B.kep);                                               \
        else                                                                                                    \
            hipLaunchKernelGGL((k_stage_ref<T, K>), grd, blk, 0, st, P, in, U, out, b, mu, B.S, B.bpart,        \
                               B.wpart, B.nmax, (const T*)B.kep);                                               \
    } while (0)
        if (kind == 1)
            M2P_REF(1);
        else if (kind == 2)
            M2P_REF(2);
        else if (kind == 3)
            M2P_REF(3);
        else
            M2P_REF(4);
#undef M2P_REF
    } else {
        dim3 blk(256), grd(sh.blocks);
        // raw buffer accesses when every byte offset of the state and the DEM
        // fits in 31 bits (4096 x 4096 FP32: 403 MB)
        const bool buf = !sh.global_addr && (uint64_t)NF * P.ny * P.pitch * sizeof(T) < (1ull << 31) &&
                         (uint64_t)(P.ny + 2 * BHALO) * P.bpitch * sizeof(T) < (1ull << 31);
#define M2P_TILED_GC(K, GH, CU, EP, WB)                                                                         \
    do {                                                                                                        \
        if (buf)                                                                                                \
            hipLaunchKernelGGL((k_stage_tiled<T, K, GH, CU, EP, true, WB>), grd, blk, 0, st, P, in, U, out, b,  \
                               mu, B.S, B.bpart, B.wpart, B.nmax, sh.R, sh.nstrips, sh.nrb);                     \
        else                                                                                                    \
            hipLaunchKernelGGL((k_stage_tiled<T, K, GH, CU, EP, false, WB>), grd, blk, 0, st, P, in, U, out, b, \
                               mu, B.S, B.bpart, B.wpart, B.nmax, sh.R, sh.nstrips, sh.nrb);                     \
    } while (0)
#define M2P_TILED(K)                                                                                            \
    do {                                                                                                        \
        const bool cu = (P.flags & kFlagCentralUpwind) != 0;                                                    \
        if (P.flags & kFlagWellBalanced)                                                                        \
            M2P_TILED_GC(K, false, false, false, true);                                                         \
        else if (P.flags & kFlagEarthPressure)                                                                  \
            M2P_TILED_GC(K, false, false, true, false);                                                         \
        else if (P.nsseg > 0) {                                                                                 \
            if (cu)                                                                                             \
                M2P_TILED_GC(K, true, true, false, false);                                                      \
            else                                                                                                \
                M2P_TILED_GC(K, true, false, false, false);                                                     \
        } else if (cu)                                                                                          \
            M2P_TILED_GC(K, false, true, false, false);                                                         \
        else                                                                                                    \
            M2P_TILED_GC(K, false, false, false, false);                                                        \
    } while (0)
        if (kind == 1)
            M2P_TILED(1);
        else if (kind == 2)
            M2P_TILED(2);
        else if (kind == 3)
            M2P_TILED(3);
        else
            M2P_TILED(4);
#undef M2P_TILED
#undef M2P_TILED_GC
    }
    return hipGetLastError();
}

template <>
int Launch<M2P_REAL>::resident_waves(const KParams& P)
{
    using T = M2P_REAL;
    int dev = 0, cus = 0, nb = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    hipError_t e;
    if (P.flags & kFlagWellBalanced)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_stage_tiled<T, 2, false, false, false, true, true>,
                                                         256, 0);
    else if (P.flags & kFlagEarthPressure)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_stage_tiled<T, 2, false, false, true>, 256, 0);
    else if (P.flags & kFlagCentralUpwind)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_stage_tiled<T, 2, false, true, false>, 256, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_stage_tiled<T, 2, false, false, false>, 256, 0);
    return e == hipSuccess ? nb * 4 * cus : 0;
}

template <>
hipError_t Launch<M2P_REAL>::init(const KParams& P, const Bufs& B, hipStream_t st)
{
    using T = M2P_REAL;
    dim3 blk(64, 4), grd((P.nx + 63) / 64, (P.ny + 3) / 4);
    hipLaunchKernelGGL((k_speeds<T>), grd, blk, 0, st, P, (const T*)B.U, (const T*)B.b, (const T*)B.mu, B.wpart);
    hipLaunchKernelGGL((k_finalize<T>), dim3(1), dim3(kFinThreads), 0, st, P, B.S, B.tables, 1, B.wpart, B.nw_ref,
                       B.bpart, B.nmax);
    return hipGetLastError();
}

template <>
hipError_t Launch<M2P_REAL>::set_state(const KParams& P, const Bufs& B, const double* f, int vertical, int has_v,
                                       hipStream_t st)
{
    using T = M2P_REAL;
    dim3 blk(64, 4), grd((P.nx + 63) / 64, (P.ny + 3) / 4);
    hipLaunchKernelGGL((k_set_state<T>), grd, blk, 0, st, P, f, vertical, has_v, (T*)B.U, (const T*)B.b);
    return hipGetLastError();
}

template <>
hipError_t Launch<M2P_REAL>::get_fields(const KParams& P, const Bufs& B, double* f, hipStream_t st)
{
    using T = M2P_REAL;
    dim3 blk(64, 4), grd((P.nx + 63) / 64, (P.ny + 3) / 4);
    hipLaunchKernelGGL((k_get_fields<T>), grd, blk, 0, st, P, (const T*)B.U, (const T*)B.b, f);
    return hipGetLastError();
}

template <>
hipError_t Launch<M2P_REAL>::mass(const KParams& P, const Bufs& B, hipStream_t st)
{
    using T = M2P_REAL;
    hipLaunchKernelGGL((k_mass<T>), dim3(kMassBlocks), dim3(256), 0, st, P, (const T*)B.U, B.mass_part);
    return hipGetLastError();
}

template <>
hipError_t Launch<M2P_REAL>::batch_part(const ScenDesc<M2P_REAL>* scen, int nscen, const int* work, int nwork, int R,
                                        int blocks, bool buf, hipStream_t st, int part, int mode)
{
    using T = M2P_REAL;
    if (part == 2) {
        hipLaunchKernelGGL((k_finalize_batch<T>), dim3(nscen), dim3(kFinThreads), 0, st, scen, mode);
        return hipGetLastError();
    }
#define M2P_BATCH(KERNEL, K)                                                                                    \
    do {                                                                                                        \
        if (buf)                                                                                                \
            hipLaunchKernelGGL((KERNEL<T, K, true>), dim3(blocks), dim3(256), 0, st, scen, work, nwork, R);     \
        else                                                                                                    \
            hipLaunchKernelGGL((KERNEL<T, K, false>), dim3(blocks), dim3(256), 0, st, scen, work, nwork, R);    \
    } while (0)
    if ((long long)blocks * 4 >= nwork) {  // one wavefront per work item
        if (part == 0)
            M2P_BATCH(k_stage_batch_flat, 1);
        else
            M2P_BATCH(k_stage_batch_flat, 2);
    } else if (part == 0)
        M2P_BATCH(k_stage_batch, 1);
    else
        M2P_BATCH(k_stage_batch, 2);
#undef M2P_BATCH
    return hipGetLastError();
}

template <>
hipError_t Launch<M2P_REAL>::jvp(const KParams& P, const Bufs& B, const void* U, const void* dU, const void* dmu,
                                 int stage, void* E, void* dE, hipStream_t st)
{
    using T = M2P_REAL;
    dim3 blk(128), grd((P.nx + 127) / 128, P.ny);
    hipLaunchKernelGGL((k_stage_jvp<T>), grd, blk, 0, st, P, (const T*)U, (const T*)dU, (const T*)B.b,
                       (const T*)B.mu, (const T*)dmu, B.S, stage, (T*)E, (T*)dE);
    return hipGetLastError();
}

template <>
hipError_t Launch<M2P_REAL>::vjp(const KParams& P, const Bufs& B, const void* U, const void* lam, double lscale,
                                 int stage, double dt, void* GT, void* DU, void* FCX, void* FCY, void* SC,
                                 void* lam_in, const void* z, double zc, void* gmu, hipStream_t st)
{
    using T = M2P_REAL;
    dim3 blk(128), grd((P.nx + 127) / 128, P.ny);
    const T* b = (const T*)B.b;
    hipLaunchKernelGGL((k_adj_post<T>), grd, blk, 0, st, P, (const T*)U, (const T*)lam, T(lscale), b,
                       (const T*)B.mu, B.S, stage, T(dt), (T*)GT, (T*)DU, (T*)gmu);
    // x-face rows 0 .. ny-1 (two wavefronts per workgroup), then y-face rows 0 .. ny
    const int nfb = std::max((adj_xwaves(P.nx) + 1) / 2, (P.nx + 127) / 128);
    hipLaunchKernelGGL((k_adj_face<T>), dim3(nfb, 2 * P.ny + 1), blk, 0, st, P, (const T*)U, (const T*)GT, b, T(dt),
                       (T*)FCX, (T*)FCY);
    hipLaunchKernelGGL((k_adj_src<T>), dim3((adj_swaves(P.nx) + 1) / 2, P.ny), blk, 0, st, P, (const T*)U,
                       (const T*)GT, b, T(dt), (T*)SC);
    // interior box (if any) and the edge ring, one launch
    const int nbx = P.nx >= 5 && P.ny >= 5 ? (P.nx - 4 + 127) / 128 : 0;
    const int nbi = nbx * (P.ny >= 5 ? P.ny - 4 : 0);
    const long long nring = adj_ring_cells(P.nx, P.ny);
    hipLaunchKernelGGL((k_adj_gather<T>), dim3((unsigned)(nbi + (nring + 1) / 2)), blk, 0, st, P, (const T*)DU,
                       (const T*)FCX, (const T*)FCY, (const T*)SC, (const T*)z, T(zc), (T*)lam_in, nbi,
                       nbx > 0 ? nbx : 1);
    return hipGetLastError();
}

template <>
hipError_t Launch<M2P_REAL>::loss(const KParams& P, const Bufs& B, const void* U, const double* target, void* lam,
                                  double* part, hipStream_t st)
{
    using T = M2P_REAL;
    hipLaunchKernelGGL((k_loss<T>), dim3(kMassBlocks), dim3(256), 0, st, P, (const T*)U, (const T*)B.b, target,
                       (T*)lam, part);
    return hipGetLastError();
}

template <>
hipError_t Launch<M2P_REAL>::dot(const KParams& P, const void* x, const void* y, double* part, hipStream_t st)
{
    using T = M2P_REAL;
    hipLaunchKernelGGL((k_dot<T>), dim3(kMassBlocks), dim3(256), 0, st, P, (const T*)x, (const T*)y, part);
    return hipGetLastError();
}

}  // namespace m2p
