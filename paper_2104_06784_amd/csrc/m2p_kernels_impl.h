// m2p_kernels_impl.h -- launchers for one precision (included by
// m2p_f64.hip / m2p_f32.hip after defining M2P_REAL).
#pragma once

#include "m2p_kernels.h"

namespace m2p {

template <>
void Launch<M2P_REAL>::grid_dims(const KParams& P, int variant, int rows, int& nbx, int& nby)
{
    (void)variant;
    (void)rows;
    nbx = (P.nx + 63) / 64;
    nby = (P.ny + 3) / 4;
}

template <>
hipError_t Launch<M2P_REAL>::step_part(const KParams& P, const Bufs& B, hipStream_t st, int variant, int rows,
                                       int part)
{
    using T = M2P_REAL;
    (void)variant;
    (void)rows;
    dim3 blk(64, 4), grd(B.nbx, B.nby);
    T* U = (T*)B.U;
    T* Us = (T*)B.Us;
    const T* b = (const T*)B.b;
    const T* mu = (const T*)B.mu;
    if (part == 0)
        hipLaunchKernelGGL((k_stage_ref<T, 1>), grd, blk, 0, st, P, U, U, Us, b, mu, B.S, B.bpart, B.nmax);
    else if (part == 1)
        hipLaunchKernelGGL((k_stage_ref<T, 2>), grd, blk, 0, st, P, Us, U, U, b, mu, B.S, B.bpart, B.nmax);
    else
        hipLaunchKernelGGL((k_finalize<T>), dim3(1), dim3(64), 0, st, P, B.S, B.bpart, B.nbx, B.nby, B.nmax,
                           B.tables, 0);
    return hipGetLastError();
}

template <>
hipError_t Launch<M2P_REAL>::init(const KParams& P, const Bufs& B, hipStream_t st)
{
    using T = M2P_REAL;
    dim3 blk(64, 4), grd((P.nx + 63) / 64, (P.ny + 3) / 4);
    hipLaunchKernelGGL((k_speeds<T>), grd, blk, 0, st, P, (const T*)B.U, (const T*)B.b, B.S);
    hipLaunchKernelGGL((k_finalize<T>), dim3(1), dim3(64), 0, st, P, B.S, B.bpart, B.nbx, B.nby, B.nmax, B.tables, 1);
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

}  // namespace m2p
