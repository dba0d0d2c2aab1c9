// m2p_adjoint.h -- tangent (JVP) and adjoint (VJP) kernels of one forward-
// Euler stage E of the scheme, for gradients of a loss through the two-step
// modified Euler method with frozen time steps.
//
// The adjoint is written as the transpose of the stage's structure:
//   out_c = Clamp(tent_c, U_c, mu_c),  tent_c = U_c + dt R_c,
//   R_c   = -(H_{c+1/2} - H_{c-1/2}) / dxi - (G_{c+1/2} - G_{c-1/2}) / deta + S_c,
// where a face flux H depends on the four cells of its reconstruction stencil
// and S_c on the cell, its four neighbours and (viscosity) its four corners.
//   pass A (cells):  cotangent of tent_c and of (U_c, mu_c) through Clamp;
//   pass B (faces):  face cotangent dt (g_R - g_L) / dxi pulled back to the
//                    four stencil cells; (cells) dt g_tent pulled back through
//                    S_c to its 34 inputs;
//   pass C (cells):  fixed-order gather of all contributions that land on a
//                    cell through the ghost-cell map (sign flips included).
// The local Jacobian-transpose products follow the structure of the forward
// arithmetic: the central flux, the face sides (side_flux), the local sources
// and the viscous face terms are reversed by hand; the Coulomb clamp,
// kappa, the desingularised quotients and the fluid-pressure products use
// forward-mode dual evaluations of the same device functions the forward
// kernels run.  Every product is the transpose of the dual-number JVP of the
// executed (FP64-order) scheme, which the tests check to 1e-12.  Non-smooth
// points (minmod, max of speeds, Coulomb stop, positivity, sqrt at 0) take the
// derivative of the branch selected by the values.
#pragma once

#include "m2p_device.h"
#include "m2p_dual.h"
#include "m2p_kernels.h"

namespace m2p {

template <typename T>
__device__ __forceinline__ Geo<Dual<T>> lift(const Geo<T>& g)
{
    Geo<Dual<T>> r;
    r.bX = Dual<T>(g.bX, T(0));
    r.bY = Dual<T>(g.bY, T(0));
    r.J = Dual<T>(g.J, T(0));
    r.c = Dual<T>(g.c, T(0));
    r.nX = Dual<T>(g.nX, T(0));
    r.nY = Dual<T>(g.nY, T(0));
    r.nZ = Dual<T>(g.nZ, T(0));
    r.A11 = Dual<T>(g.A11, T(0));
    r.A12 = Dual<T>(g.A12, T(0));
    r.A21 = Dual<T>(g.A21, T(0));
    r.A22 = Dual<T>(g.A22, T(0));
    return r;
}

template <typename T> __device__ __forceinline__ Geo<T> liftg(const Geo<T>& g, T*) { return g; }
template <typename T> __device__ __forceinline__ Geo<Dual<T>> liftg(const Geo<T>& g, Dual<T>*) { return lift(g); }
template <typename T> __device__ __forceinline__ T liftv(T x, T*) { return x; }
template <typename T> __device__ __forceinline__ Dual<T> liftv(T x, Dual<T>*) { return Dual<T>(x, T(0)); }

// Geometry of the five cells a stage at (i, j) needs, in the base type.
template <typename T>
struct Geo5 {
    Geo<T> C, W, E, S, N;
};

template <typename T>
__device__ __forceinline__ Geo5<T> geo5(const KParams& P, const T* __restrict__ b, int i, int j)
{
    const Consts<T> K(P);
    auto bv = [&](int ii, int jj) { return b[(size_t)(jj + BHALO) * P.bpitch + BOFF + ii]; };
    auto g = [&](int ii, int jj) {
        return geometry(bv(ii + 1, jj), bv(ii - 1, jj), bv(ii, jj + 1), bv(ii, jj - 1), K.two_dxi, K.two_deta);
    };
    Geo5<T> r;
    r.C = g(i, j);
    r.W = g(i - 1, j);
    r.E = g(i + 1, j);
    r.S = g(i, j - 1);
    r.N = g(i, j + 1);
    return r;
}

// Stencil values of a cell: row i-2..i+2, column j-2..j+2, 3x3 box.
template <typename TT>
struct Stencil {
    TT row[5][NF], col[5][NF], box[3][3][NF];
};

// Ghost-mapped load of one cell's 6 fields (base type).
template <typename T>
__device__ __forceinline__ void load_mapped(const KParams& P, const T* __restrict__ U, int ii, int jj, T u[NF])
{
    const size_t fs = (size_t)P.ny * P.pitch;
    int fx = 0, fy = 0;
    const int mi = map_index(ii, P.nx, P.bc[0], P.bc[1], fx);
    const int mj = map_index(jj, P.ny, P.bc[2], P.bc[3], fy);
    const size_t c = (size_t)mj * P.pitch + mi;
#pragma unroll
    for (int k = 0; k < NF; k++) u[k] = U[k * fs + c];
    if (fx) {
        u[1] = -u[1];
        u[4] = -u[4];
    }
    if (fy) {
        u[2] = -u[2];
        u[5] = -u[5];
    }
}

// Sources (all but the Coulomb clamp) of a cell, including viscosity, from its
// stencil: returns the per-component source vector added to R (mass: 0) and
// the Src record (kappa_s for the clamp).
template <typename TT, typename T>
__device__ __forceinline__ void cell_sources(const KParams& P, const Consts<TT>& K, const Stencil<TT>& s,
                                             const Geo5<T>& g5, Src<TT>& Sr, TT& svx, TT& svy)
{
    TT* tag = nullptr;
    const Geo<TT> gC = liftg(g5.C, tag), gW = liftg(g5.W, tag), gE = liftg(g5.E, tag), gS = liftg(g5.S, tag),
                  gN = liftg(g5.N, tag);
    const T two_dxi = T(P.two_dxi), two_deta = T(P.two_deta);
    TT dn[6];
    dn[0] = liftv((g5.E.nX - g5.W.nX) / two_dxi, tag);
    dn[1] = liftv((g5.E.nY - g5.W.nY) / two_dxi, tag);
    dn[2] = liftv((g5.E.nZ - g5.W.nZ) / two_dxi, tag);
    dn[3] = liftv((g5.N.nX - g5.S.nX) / two_deta, tag);
    dn[4] = liftv((g5.N.nY - g5.S.nY) / two_deta, tag);
    dn[5] = liftv((g5.N.nZ - g5.S.nZ) / two_deta, tag);
    const TT dGx = (fluid_G(s.row[3][0], s.row[3][3], gE) - fluid_G(s.row[1][0], s.row[1][3], gW)) / K.two_dxi;
    const TT dGy = (fluid_G(s.col[3][0], s.col[3][3], gN) - fluid_G(s.col[1][0], s.col[1][3], gS)) / K.two_deta;
    sources(K, P.flags, s.row[2], gC, dn, dGx, dGy, Sr);
    svx = TT(0.0);
    svy = TT(0.0);
    if (P.visc) {
        TT u9[3][3], w9[3][3];
        for (int a = 0; a < 3; a++)
            for (int c = 0; c < 3; c++) {
                u9[a][c] = dsg(s.box[a][c][4], s.box[a][c][3], K.md);
                w9[a][c] = dsg(s.box[a][c][5], s.box[a][c][3], K.md);
            }
        const TT JhC = s.row[2][0] + s.row[2][3];
        const TT JhW = s.row[1][0] + s.row[1][3], JhE = s.row[3][0] + s.row[3][3];
        const TT JhS = s.col[1][0] + s.col[1][3], JhN = s.col[3][0] + s.col[3][3];
        TT cyu[3], cyw[3], cxu[3], cxw[3];
        for (int q = 0; q < 3; q++) {
            cyu[q] = cdiff(u9[2][q], u9[0][q], K.deta);
            cyw[q] = cdiff(w9[2][q], w9[0][q], K.deta);
            cxu[q] = cdiff(u9[q][2], u9[q][0], K.dxi);
            cxw[q] = cdiff(w9[q][2], w9[q][0], K.dxi);
        }
        TT FX0, FY0, FX1, FY1, GX0, GY0, GX1, GY1;
        visc_xface_c(u9[1][0], w9[1][0], u9[1][1], w9[1][1], cyu[0], cyw[0], cyu[1], cyw[1], JhW, JhC, gW, gC, K.dxi,
                     FX0, FY0);
        visc_xface_c(u9[1][1], w9[1][1], u9[1][2], w9[1][2], cyu[1], cyw[1], cyu[2], cyw[2], JhC, JhE, gC, gE, K.dxi,
                     FX1, FY1);
        visc_yface_c(u9[0][1], w9[0][1], u9[1][1], w9[1][1], cxu[0], cxw[0], cxu[1], cxw[1], JhS, JhC, gS, gC,
                     K.deta, GX0, GY0);
        visc_yface_c(u9[1][1], w9[1][1], u9[2][1], w9[2][1], cxu[1], cxw[1], cxu[2], cxw[2], JhC, JhN, gC, gN,
                     K.deta, GX1, GY1);
        const TT SvX = (FX1 - FX0) / K.dxi + (GX1 - GX0) / K.deta;
        const TT SvY = (FY1 - FY0) / K.dxi + (GY1 - GY0) / K.deta;
        svx = K.eps * Sr.phif * K.inv_n_r * SvX;
        svy = K.eps * Sr.phif * K.inv_n_r * SvY;
    }
}

// Face flux H_{a+1/2} in direction d from the 4-cell window (a-1 .. a+2) and
// the geometries of cells a and a+1.
template <typename TT, typename T>
__device__ __forceinline__ void face_flux(const Consts<TT>& K, const TT w[4][NF], const Geo<T>& ga, const Geo<T>& gb,
                                          int d, TT H[NF])
{
    TT* tag = nullptr;
    TT uL[NF], uR[NF];
#pragma unroll
    for (int k = 0; k < NF; k++) {
        const TT s0 = minmod(w[1][k] - w[0][k], w[2][k] - w[1][k]);
        const TT s1 = minmod(w[2][k] - w[1][k], w[3][k] - w[2][k]);
        uL[k] = w[1][k] + TT(0.5) * s0;
        uR[k] = w[2][k] - TT(0.5) * s1;
    }
    central_flux(K, uL, liftg(ga, tag), uR, liftg(gb, tag), d, H);
}

// Whole stage at interior cell (i, j) from its stencil (the arithmetic of the
// forward kernels): tentative update and clamped output.
template <typename TT, typename T>
__device__ __forceinline__ void cell_stage(const KParams& P, const Stencil<TT>& s, const Geo5<T>& g5, TT dt, TT tmu,
                                           const double (*inf)[4], int i, int j, TT tent[NF], TT out[NF])
{
    const Consts<TT> K(P);
    TT* tag = nullptr;
    TT HXl[NF], HXr[NF], HYb[NF], HYt[NF], w[4][NF];
    for (int q = 0; q < 4; q++)
        for (int k = 0; k < NF; k++) w[q][k] = s.row[q][k];
    face_flux(K, w, g5.W, g5.C, 0, HXl);
    for (int q = 0; q < 4; q++)
        for (int k = 0; k < NF; k++) w[q][k] = s.row[q + 1][k];
    face_flux(K, w, g5.C, g5.E, 0, HXr);
    for (int q = 0; q < 4; q++)
        for (int k = 0; k < NF; k++) w[q][k] = s.col[q][k];
    face_flux(K, w, g5.S, g5.C, 1, HYb);
    for (int q = 0; q < 4; q++)
        for (int k = 0; k < NF; k++) w[q][k] = s.col[q + 1][k];
    face_flux(K, w, g5.C, g5.N, 1, HYt);
    const Geo<TT> gC = liftg(g5.C, tag);
    int sgi;
    if (i == 0 && (sgi = inflow_seg_at(P, 0, j)) >= 0)
        inflow_flux(K, gC, 0, +1, TT(inf[sgi][0]), TT(inf[sgi][1]), TT(inf[sgi][2]), TT(inf[sgi][3]), HXl);
    if (i == P.nx - 1 && (sgi = inflow_seg_at(P, 1, j)) >= 0)
        inflow_flux(K, gC, 0, -1, TT(inf[sgi][0]), TT(inf[sgi][1]), TT(inf[sgi][2]), TT(inf[sgi][3]), HXr);
    if (j == 0 && (sgi = inflow_seg_at(P, 2, i)) >= 0)
        inflow_flux(K, gC, 1, +1, TT(inf[sgi][0]), TT(inf[sgi][1]), TT(inf[sgi][2]), TT(inf[sgi][3]), HYb);
    if (j == P.ny - 1 && (sgi = inflow_seg_at(P, 3, i)) >= 0)
        inflow_flux(K, gC, 1, -1, TT(inf[sgi][0]), TT(inf[sgi][1]), TT(inf[sgi][2]), TT(inf[sgi][3]), HYt);
    Src<TT> Sr;
    TT svx, svy;
    cell_sources(P, K, s, g5, Sr, svx, svy);
    tentative(K, s.row[2], HXl, HXr, HYb, HYt, Sr, svx, svy, dt, tent);
    for (int k = 0; k < NF; k++) out[k] = tent[k];
    clamp_cell(K, gC, Sr.kappa_s, dt, tmu, out);
}

template <typename T>
__device__ __forceinline__ void load_stencil(const KParams& P, const T* __restrict__ U, int i, int j, Stencil<T>& s)
{
    for (int q = 0; q < 5; q++) load_mapped(P, U, i - 2 + q, j, s.row[q]);
    for (int q = 0; q < 5; q++) load_mapped(P, U, i, j - 2 + q, s.col[q]);
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) load_mapped(P, U, i - 1 + c, j - 1 + a, s.box[a][c]);
}

// ---------------------------------------------------------------- JVP / E

// E(U) and its directional derivative along dU (both [6][ny][pitch]).
template <typename T>
__global__ void __launch_bounds__(128) k_stage_jvp(KParams P, const T* __restrict__ U, const T* __restrict__ dU,
                                                   const T* __restrict__ b, const T* __restrict__ mu,
                                                   const T* __restrict__ dmu, const DevScalars* __restrict__ S,
                                                   int stage, T* __restrict__ E, T* __restrict__ dE)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= P.nx) return;
    using TT = Dual<T>;
    Stencil<T> s0, s1;
    load_stencil(P, U, i, j, s0);
    load_stencil(P, dU, i, j, s1);
    Stencil<TT> s;
    for (int q = 0; q < 5; q++)
        for (int k = 0; k < NF; k++) {
            s.row[q][k] = TT(s0.row[q][k], s1.row[q][k]);
            s.col[q][k] = TT(s0.col[q][k], s1.col[q][k]);
        }
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++)
            for (int k = 0; k < NF; k++) s.box[a][c][k] = TT(s0.box[a][c][k], s1.box[a][c][k]);
    const Geo5<T> g5 = geo5(P, b, i, j);
    const size_t c = (size_t)j * P.pitch + i, fs = (size_t)P.ny * P.pitch;
    const TT tmu(P.has_mu ? mu[c] : T(P.tan_d), dmu ? dmu[c] : T(0));
    TT tent[NF], out[NF];
    cell_stage(P, s, g5, TT(T(S->dt), T(0)), tmu, S->inflow[stage], i, j, tent, out);
    for (int k = 0; k < NF; k++) {
        E[k * fs + c] = out[k].v;
        dE[k * fs + c] = out[k].d;
    }
}

// ---------------------------------------------------------------- adjoint

// Pass A: per cell, the cotangent of the tentative state (GT), the direct
// cotangent of U_c (identity of the update + clamp through kappa_s) into DU,
// and the friction-field cotangent (accumulated into gmu).  The incoming
// cotangent is lscale * lam (the Heun average passes half of it to the second
// stage).
template <typename T>
__global__ void __launch_bounds__(128) k_adj_post(KParams P, const T* __restrict__ U, const T* __restrict__ lam,
                                                  T lscale, const T* __restrict__ b, const T* __restrict__ mu,
                                                  const DevScalars* __restrict__ S, int stage, T dt,
                                                  T* __restrict__ GT, T* __restrict__ DU, T* __restrict__ gmu)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= P.nx) return;
    const size_t c = (size_t)j * P.pitch + i, fs = (size_t)P.ny * P.pitch;
    Stencil<T> s;
    load_stencil(P, U, i, j, s);
    const Geo5<T> g5 = geo5(P, b, i, j);
    const T tmu = P.has_mu ? mu[c] : T(P.tan_d);
    T tent[NF], out[NF];
    cell_stage(P, s, g5, dt, tmu, S->inflow[stage], i, j, tent, out);
    T lo[NF];
    for (int k = 0; k < NF; k++) lo[k] = lscale * lam[k * fs + c];
    using TT = Dual<T>;
    const Consts<TT> K(P);
    const Geo<TT> gC = lift(g5.C);
    const T two_dxi = T(P.two_dxi), two_deta = T(P.two_deta);
    TT dn[6];
    dn[0] = TT((g5.E.nX - g5.W.nX) / two_dxi, T(0));
    dn[1] = TT((g5.E.nY - g5.W.nY) / two_dxi, T(0));
    dn[2] = TT((g5.E.nZ - g5.W.nZ) / two_dxi, T(0));
    dn[3] = TT((g5.N.nX - g5.S.nX) / two_deta, T(0));
    dn[4] = TT((g5.N.nY - g5.S.nY) / two_deta, T(0));
    dn[5] = TT((g5.N.nZ - g5.S.nZ) / two_deta, T(0));
    // clamp inputs: tentative state (6), kappa_s, friction; kappa_s depends on
    // the cell's own solid fields only
    const T* uc = s.row[2];
    auto kappa_s = [&](int d) {
        const TT ms(uc[0], d == 0 ? T(1) : T(0));
        return kappa_of(dsg(TT(uc[1], d == 1 ? T(1) : T(0)), ms, K.md), dsg(TT(uc[2], d == 2 ? T(1) : T(0)), ms, K.md),
                        gC, dn);
    };
    const T kap_s = kappa_s(-1).v;
    T gcl[8];
    for (int d = 0; d < 8; d++) {
        TT o[NF];
        for (int k = 0; k < NF; k++) o[k] = TT(tent[k], d == k ? T(1) : T(0));
        clamp_cell(K, gC, TT(kap_s, d == 6 ? T(1) : T(0)), TT(dt, T(0)), TT(tmu, d == 7 ? T(1) : T(0)), o);
        T acc = T(0);
        for (int k = 0; k < NF; k++) acc += lo[k] * o[k].d;
        gcl[d] = acc;
    }
    T g[13];
    for (int k = 0; k < NF; k++) g[k] = gcl[k];
    g[12] = gcl[7];
    for (int d = 0; d < NF; d++) g[6 + d] = d < 3 ? gcl[6] * kappa_s(d).d : T(0);
    for (int k = 0; k < NF; k++) {
        GT[k * fs + c] = g[k];
        DU[k * fs + c] = g[k] + g[6 + k];
    }
    gmu[c] += g[12];
}

// Partial derivatives of dsg(num, den, md) with respect to num and den (dual
// evaluations of the same function).
template <typename T>
__device__ __forceinline__ void dsg_partials(T num, T den, T md, T& d_num, T& d_den)
{
    using TT = Dual<T>;
    d_num = dsg(TT(num, T(1)), TT(den, T(0)), TT(md, T(0))).d;
    d_den = dsg(TT(num, T(0)), TT(den, T(1)), TT(md, T(0))).d;
}

// Which argument the (dual) minmod selects: 0 the first, 1 the second, 2
// neither (result 0).  Mirrors the selects of minmod on dual numbers.
template <typename T>
__device__ __forceinline__ int minmod_pick(T a, T b)
{
    const bool pos = (int)(a > T(0)) & (int)(b > T(0));
    const bool neg = (int)(a < T(0)) & (int)(b < T(0));
    if (pos) return a < b ? 0 : 1;
    if (neg) return a > b ? 0 : 1;
    return 2;
}

// Transpose of one reconstructed side: cotangents of its flux F, conserved
// values q and phase speeds a pulled back to the side's six conserved values
// (the generic side_flux, reverse sweep written out; the desingularised
// quotients through dual evaluations of dsg).
template <typename T>
__device__ __forceinline__ void side_flux_vjp(const Consts<T>& K, const T u[NF], const Geo<T>& g, int d,
                                              const T lF[NF], const T lq[NF], const T la[2], T lu[NF])
{
    // forward values
    const T ms = u[0], mf = u[3];
    const T hs = ms / g.J, hf = mf / g.J, h = hs + hf;
    const T vXs = dsg(u[1], ms, K.md), vYs = dsg(u[2], ms, K.md);
    const T vXf = dsg(u[4], mf, K.md), vYf = dsg(u[5], mf, K.md);
    const T Ns = g.c * (T(1) - K.al) * hs / T(2);
    const T pf = g.c * h / T(2);
    const T Ax = d == 0 ? g.A11 : g.A21;
    const T Ay = d == 0 ? g.A12 : g.A22;
    const T Ann = d == 0 ? g.A11 : g.A22;
    const T vns = d == 0 ? vXs : vYs;
    const T vnf = d == 0 ? vXf : vYf;
    const T eJ = K.eps * g.J;
    const T cs = K.eps * Ann * g.c * (T(1) - K.al) * (h + hs) / T(2);
    const T cf = K.eps * Ann * g.c * h;
    // speeds |v_n| + sqrt(max(c, 0)); sqrt has derivative 0 at 0
    T vns_b = la[0] * (vns < T(0) ? T(-1) : T(1));
    T vnf_b = la[1] * (vnf < T(0) ? T(-1) : T(1));
    const T rs = cs > T(0) ? ::sqrt(cs) : T(0), rf = cf > T(0) ? ::sqrt(cf) : T(0);
    const T cs_b = rs > T(0) ? la[0] / (T(2) * rs) : T(0);
    const T cf_b = rf > T(0) ? la[1] / (T(2) * rf) : T(0);
    const T kcs = K.eps * Ann * g.c * (T(1) - K.al) / T(2);
    T h_b = cs_b * kcs + cf_b * (K.eps * Ann * g.c);
    T hs_b = cs_b * kcs;
    // conserved values q
    T ms_b = lq[0] + lq[1] * vXs + lq[2] * vYs, mf_b = lq[3] + lq[4] * vXf + lq[5] * vYf;
    T vXs_b = lq[1] * ms, vYs_b = lq[2] * ms, vXf_b = lq[4] * mf, vYf_b = lq[5] * mf;
    // advective parts m v_a v_n
    ms_b += lF[0] * vns + (lF[1] * vXs + lF[2] * vYs) * vns;
    vns_b += lF[0] * ms + (lF[1] * vXs + lF[2] * vYs) * ms;
    vXs_b += lF[1] * ms * vns;
    vYs_b += lF[2] * ms * vns;
    mf_b += lF[3] * vnf + (lF[4] * vXf + lF[5] * vYf) * vnf;
    vnf_b += lF[3] * mf + (lF[4] * vXf + lF[5] * vYf) * mf;
    vXf_b += lF[4] * mf * vnf;
    vYf_b += lF[5] * mf * vnf;
    // pressure parts eps J_b h A N^s and eps J_b h A pbar^f
    const T ws = lF[1] * Ax + lF[2] * Ay, wf = lF[4] * Ax + lF[5] * Ay;
    h_b += eJ * (ws * Ns + wf * pf);
    const T Ns_b = eJ * h * ws, pf_b = eJ * h * wf;
    hs_b += Ns_b * g.c * (T(1) - K.al) / T(2);
    h_b += pf_b * g.c / T(2);
    if (d == 0) {
        vXs_b += vns_b;
        vXf_b += vnf_b;
    } else {
        vYs_b += vns_b;
        vYf_b += vnf_b;
    }
    hs_b += h_b;
    const T hf_b = h_b;
    ms_b += hs_b / g.J;
    mf_b += hf_b / g.J;
    T dn_, dd_;
    dsg_partials(u[1], ms, K.md, dn_, dd_);
    lu[1] = vXs_b * dn_;
    ms_b += vXs_b * dd_;
    dsg_partials(u[2], ms, K.md, dn_, dd_);
    lu[2] = vYs_b * dn_;
    ms_b += vYs_b * dd_;
    dsg_partials(u[4], mf, K.md, dn_, dd_);
    lu[4] = vXf_b * dn_;
    mf_b += vXf_b * dd_;
    dsg_partials(u[5], mf, K.md, dn_, dd_);
    lu[5] = vYf_b * dn_;
    mf_b += vYf_b * dd_;
    lu[0] = ms_b;
    lu[3] = mf_b;
}

// Transpose of the face flux H(w) of face_flux: cotangent gH of H pulled back
// to the 24 stencil values w[4][NF] (out[6 q + k]).  Central flux by hand
// (H = (F_L + F_R)/2 - a/2 (q_R - q_L), a = max of the side speeds per
// phase), each side through side_flux_vjp, then the reconstruction through
// the branch minmod selects -- the same linear map as dual evaluations of
// face_flux along the 24 unit directions.
template <typename T>
__device__ __forceinline__ void face_flux_vjp(const KParams& P, const T w[4][NF], const Geo<T>& ga, const Geo<T>& gb,
                                              int d, const T gH[NF], T out[24])
{
    const Consts<T> Kb(P);
    T uL[NF], uR[NF];
    int p0[NF], p1[NF];
#pragma unroll
    for (int k = 0; k < NF; k++) {
        const T a0 = w[1][k] - w[0][k], b0 = w[2][k] - w[1][k], b1 = w[3][k] - w[2][k];
        p0[k] = minmod_pick(a0, b0);
        p1[k] = minmod_pick(b0, b1);
        uL[k] = w[1][k] + T(0.5) * minmod(a0, b0);
        uR[k] = w[2][k] - T(0.5) * minmod(b0, b1);
    }
    // side values (the flux, conserved values and speeds of each side)
    T FL[NF], FR[NF], qL[NF], qR[NF], aL[2], aR[2];
    side_flux(Kb, uL, ga, d, FL, qL, aL);
    side_flux(Kb, uR, gb, d, FR, qR, aR);
    T lF[NF], lqL[NF], lqR[NF], laL[2], laR[2];
#pragma unroll
    for (int ph = 0; ph < 2; ph++) {
        const bool left = aL[ph] > aR[ph];
        const T am = left ? aL[ph] : aR[ph];
        T la = T(0);
#pragma unroll
        for (int k = 3 * ph; k < 3 * ph + 3; k++) {
            lF[k] = T(0.5) * gH[k];
            lqL[k] = T(0.5) * am * gH[k];
            lqR[k] = -(T(0.5) * am * gH[k]);
            la += gH[k] * (qR[k] - qL[k]);
        }
        la = -(T(0.5) * la);
        laL[ph] = left ? la : T(0);
        laR[ph] = left ? T(0) : la;
    }
    T luL[NF], luR[NF];
    side_flux_vjp(Kb, uL, ga, d, lF, lqL, laL, luL);
    side_flux_vjp(Kb, uR, gb, d, lF, lqR, laR, luR);
    T lw[4][NF];
#pragma unroll
    for (int q = 0; q < 4; q++)
#pragma unroll
        for (int k = 0; k < NF; k++) lw[q][k] = T(0);
#pragma unroll
    for (int k = 0; k < NF; k++) {
        // uL = w1 + s0 / 2, s0 = minmod(w1 - w0, w2 - w1)
        lw[1][k] += luL[k];
        const T ls0 = T(0.5) * luL[k];
        if (p0[k] == 0) {
            lw[1][k] += ls0;
            lw[0][k] -= ls0;
        } else if (p0[k] == 1) {
            lw[2][k] += ls0;
            lw[1][k] -= ls0;
        }
        // uR = w2 - s1 / 2, s1 = minmod(w2 - w1, w3 - w2)
        lw[2][k] += luR[k];
        const T ls1 = -(T(0.5) * luR[k]);
        if (p1[k] == 0) {
            lw[2][k] += ls1;
            lw[1][k] -= ls1;
        } else if (p1[k] == 1) {
            lw[3][k] += ls1;
            lw[2][k] -= ls1;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; q++)
#pragma unroll
        for (int k = 0; k < NF; k++) out[6 * q + k] = lw[q][k];
}

// The 24 stencil cotangents of one face (out[6 q + k] for cell a-1+q, a the
// face's left cell): x-face (d = 0) between (i, j) and (i + 1, j), y-face
// (d = 1) between (i, j) and (i, j + 1).  Faces with a prescribed inflow flux
// do not depend on the state: zeros.
template <typename T>
__device__ __forceinline__ void adj_face_out(const KParams& P, const T* __restrict__ U, const T* __restrict__ GT,
                                             const T* __restrict__ b, int d, T dt, int i, int j, T out[24])
{
    const size_t fs = (size_t)P.ny * P.pitch;
    bool fixed = false;
    if (d == 0 && i == -1) fixed = inflow_seg_at(P, 0, j) >= 0;
    if (d == 0 && i == P.nx - 1) fixed = fixed || inflow_seg_at(P, 1, j) >= 0;
    if (d == 1 && j == -1) fixed = inflow_seg_at(P, 2, i) >= 0;
    if (d == 1 && j == P.ny - 1) fixed = fixed || inflow_seg_at(P, 3, i) >= 0;
    if (fixed) {
        for (int q = 0; q < 24; q++) out[q] = T(0);
        return;
    }
    // face cotangent: R_left has -H/h, R_right has +H/h
    const int li = i, lj = j, ri = d == 0 ? i + 1 : i, rj = d == 0 ? j : j + 1;
    const T h = T(d == 0 ? P.dxi : P.deta);
    T gH[NF];
    for (int k = 0; k < NF; k++) {
        const T gl = (li >= 0 && lj >= 0) ? GT[k * fs + (size_t)lj * P.pitch + li] : T(0);
        const T gr = (ri < P.nx && rj < P.ny) ? GT[k * fs + (size_t)rj * P.pitch + ri] : T(0);
        gH[k] = dt * (gr - gl) / h;
    }
    T w0[4][NF];
    for (int q = 0; q < 4; q++) {
        const int ci = d == 0 ? i - 1 + q : i, cj = d == 0 ? j : j - 1 + q;
        load_mapped(P, U, ci, cj, w0[q]);
    }
    const Consts<T> Kb(P);
    auto bv = [&](int ii, int jj) { return b[(size_t)(jj + BHALO) * P.bpitch + BOFF + ii]; };
    auto geo = [&](int ii, int jj) {
        return geometry(bv(ii + 1, jj), bv(ii - 1, jj), bv(ii, jj + 1), bv(ii, jj - 1), Kb.two_dxi, Kb.two_deta);
    };
    const Geo<T> ga = geo(li, lj), gb = geo(ri, rj);
    face_flux_vjp(P, w0, ga, gb, d, gH, out);
}

// Wavefronts of x-faces per grid row: each covers 60 cells of the row
// extended by two ghost columns per side (extended column e = i + 2).
__host__ __device__ inline int adj_xwaves(int nx) { return (nx + 4 + 59) / 60; }

// Pass B, faces, in one launch of 128-thread workgroups.  Grid rows
// 0 .. ny-1: x-faces of grid row j, gathered per cell in registers -- lane l
// of wavefront w computes face f = 60 w - 4 + l (between cells f and f + 1;
// faces outside [-1, nx-1] contribute zeros) and lanes 1..60 sum the four
// faces of cell f + 1 (slots 3, 2, 1, 0 of faces f - 1 .. f + 2, fixed
// order) into XS[6][ny][nx + 4] at extended column f + 3, ghost columns
// included.  Grid rows ny .. 2 ny: y-faces j in [-1, ny-1], one thread per
// face, 24 stencil cotangents into FCY[24][faces] (slot-major; slot = 6 *
// cell + field, cells j-1 .. j+2).
template <typename T>
__global__ void __launch_bounds__(128) k_adj_face(KParams P, const T* __restrict__ U, const T* __restrict__ GT,
                                                  const T* __restrict__ b, T dt, T* __restrict__ XS,
                                                  T* __restrict__ FCY)
{
    T out[24];
    if ((int)blockIdx.y < P.ny) {
        const int j = (int)blockIdx.y;
        const int lane = threadIdx.x & 63;
        const int w = (int)blockIdx.x * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6);
        if (w >= adj_xwaves(P.nx)) return;  // whole wavefront
        const int f = 60 * w - 4 + lane;
        if (f >= -1 && f <= P.nx - 1)
            adj_face_out(P, U, GT, b, 0, dt, f, j, out);
        else
            for (int q = 0; q < 24; q++) out[q] = T(0);
        // every lane of the wavefront takes part in the shuffles
        T acc[NF];
#pragma unroll
        for (int k = 0; k < NF; k++) {
            const T a3 = __shfl(out[18 + k], lane - 1, 64);
            const T a1 = __shfl(out[6 + k], lane + 1, 64);
            const T a0 = __shfl(out[k], lane + 2, 64);
            acc[k] = ((a3 + out[12 + k]) + a1) + a0;
        }
        const int e = f + 3;
        if (lane >= 1 && lane <= 60 && e < P.nx + 4) {
            const size_t nxs = (size_t)P.ny * (P.nx + 4), o = (size_t)j * (P.nx + 4) + e;
#pragma unroll
            for (int k = 0; k < NF; k++) XS[k * nxs + o] = acc[k];
        }
        return;
    }
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P.nx) return;
    const int line = (int)blockIdx.y - P.ny;  // face row: the face between rows line - 1 and line
    adj_face_out(P, U, GT, b, 1, dt, t, line - 1, out);
    const size_t fidx = (size_t)line * P.nx + t, nfaces = (size_t)P.nx * (P.ny + 1);
    for (int q = 0; q < 24; q++) FCY[q * nfaces + fidx] = out[q];
}

// Source input slots: 0..5 centre fields; 6..21 neighbour (E, W, N, S) x
// fields (0, 3, 4, 5); 22..33 corner (NE, NW, SE, SW) x fields (3, 4, 5).
__device__ __forceinline__ void src_slot(int s, int& di, int& dj, int& k)
{
    if (s < 6) {
        di = 0;
        dj = 0;
        k = s;
        return;
    }
    if (s < 22) {
        const int n = (s - 6) / 4, f = (s - 6) % 4;
        const int odi[4] = {1, -1, 0, 0}, odj[4] = {0, 0, 1, -1};
        const int fk[4] = {0, 3, 4, 5};
        di = odi[n];
        dj = odj[n];
        k = fk[f];
        return;
    }
    const int n = (s - 22) / 3, f = (s - 22) % 3;
    const int odi[4] = {1, -1, 1, -1}, odj[4] = {1, 1, -1, -1};
    di = odi[n];
    dj = odj[n];
    k = 3 + f;
}

// Reverse sweep of the generic sources() at one cell: cotangents L[ph][a] of
// the momentum sources (the sums sn + sf + sv (+ sd) that enter the update)
// and Lphif of phi^f pulled back to the cell's six fields (ubar) and to the
// two fluid-pressure gradients.  Same linear map as dual evaluations of
// sources() along the eight unit directions, in one pass.
template <typename T>
__device__ __forceinline__ void sources_vjp(const Consts<T>& K, int flags, const T u[NF], const Geo<T>& g,
                                            const T dn[6], T dGx, T dGy, const T L[2][2], T Lphif, T ubar[NF],
                                            T& dGx_bar, T& dGy_bar)
{
    using TT = Dual<T>;
    // forward values (the arithmetic of the generic sources())
    const T ms = u[0], mf = u[3];
    const T hs = ms / g.J, hf = mf / g.J, h = hs + hf;
    const T mt = ms + mf;
    const T phis = dsg(ms, mt, K.md), phif = dsg(mf, mt, K.md);
    const T v00 = dsg(u[1], ms, K.md), v01 = dsg(u[2], ms, K.md);
    const T v10 = dsg(u[4], mf, K.md), v11 = dsg(u[5], mf, K.md);
    const T kap0 = kappa_of(v00, v01, g, dn), kap1 = kappa_of(v10, v11, g, dn);
    const T fs_ = g.c * (T(1) - K.al) - K.eps_chi * kap0, ff_ = g.c - K.eps_chi * kap1;
    const T pbs = hs * fs_, pbf = hf * ff_;
    const T gx = g.A11 * dGx + g.A21 * dGy, gy = g.A12 * dGx + g.A22 * dGy;
    const T wf = (flags & 1) ? phif : phis;
    const T Kd = g.J * K.c_d * phis * phif * h;
    const T dv0 = v10 - v00, dv1 = v11 - v01;
    const T fr = g.J * phif * h * K.theta_b * K.inv_n_r / K.eps;
    // s_n = J p_b n (horizontal), p_b clamped at 0
    const T pbs_bar = pbs < T(0) ? T(0) : L[0][0] * g.J * g.nX + L[0][1] * g.J * g.nY;
    const T pbf_bar = pbf < T(0) ? T(0) : L[1][0] * g.J * g.nX + L[1][1] * g.J * g.nY;
    T hs_bar = pbs_bar * fs_, hf_bar = pbf_bar * ff_, h_bar = T(0);
    const T kap0_bar = -(pbs_bar * hs * K.eps_chi), kap1_bar = -(pbf_bar * hf * K.eps_chi);
    // s_f: -eps alpha phi^s grad G (solid), eps w^f grad G (fluid)
    T phis_bar = -(K.eps * K.al) * (gx * L[0][0] + gy * L[0][1]);
    const T wf_bar = K.eps * (gx * L[1][0] + gy * L[1][1]);
    T phif_bar = Lphif;
    if (flags & 1)
        phif_bar += wf_bar;
    else
        phis_bar += wf_bar;
    const T gx_bar = -(K.eps * K.al * phis) * L[0][0] + K.eps * wf * L[1][0];
    const T gy_bar = -(K.eps * K.al * phis) * L[0][1] + K.eps * wf * L[1][1];
    dGx_bar = g.A11 * gx_bar + g.A12 * gy_bar;
    dGy_bar = g.A21 * gx_bar + g.A22 * gy_bar;
    // s_v: alpha Kd (v^f - v^s) (solid), -Kd (v^f - v^s) (fluid)
    const T Kd_bar = (K.al * L[0][0] - L[1][0]) * dv0 + (K.al * L[0][1] - L[1][1]) * dv1;
    const T dv0_bar = (K.al * L[0][0] - L[1][0]) * Kd, dv1_bar = (K.al * L[0][1] - L[1][1]) * Kd;
    T v00_bar = -dv0_bar, v01_bar = -dv1_bar, v10_bar = dv0_bar, v11_bar = dv1_bar;
    phis_bar += Kd_bar * g.J * K.c_d * phif * h;
    phif_bar += Kd_bar * g.J * K.c_d * phis * h;
    h_bar += Kd_bar * g.J * K.c_d * phis * phif;
    // s_d^f: -fr v^f
    const T fr_bar = -(v10 * L[1][0] + v11 * L[1][1]);
    v10_bar -= fr * L[1][0];
    v11_bar -= fr * L[1][1];
    phif_bar += fr_bar * g.J * h * K.theta_b * K.inv_n_r / K.eps;
    h_bar += fr_bar * g.J * phif * K.theta_b * K.inv_n_r / K.eps;
    // kappa of each phase through its velocities
    const Geo<TT> gd = lift(g);
    TT dnd[6];
#pragma unroll
    for (int q = 0; q < 6; q++) dnd[q] = TT(dn[q], T(0));
    v00_bar += kap0_bar * kappa_of(TT(v00, T(1)), TT(v01, T(0)), gd, dnd).d;
    v01_bar += kap0_bar * kappa_of(TT(v00, T(0)), TT(v01, T(1)), gd, dnd).d;
    v10_bar += kap1_bar * kappa_of(TT(v10, T(1)), TT(v11, T(0)), gd, dnd).d;
    v11_bar += kap1_bar * kappa_of(TT(v10, T(0)), TT(v11, T(1)), gd, dnd).d;
    // thicknesses and desingularised quotients
    hs_bar += h_bar;
    hf_bar += h_bar;
    T ms_bar = hs_bar / g.J, mf_bar = hf_bar / g.J, mt_bar = T(0);
    T dn_, dd_;
    dsg_partials(ms, mt, K.md, dn_, dd_);
    ms_bar += phis_bar * dn_;
    mt_bar += phis_bar * dd_;
    dsg_partials(mf, mt, K.md, dn_, dd_);
    mf_bar += phif_bar * dn_;
    mt_bar += phif_bar * dd_;
    ms_bar += mt_bar;
    mf_bar += mt_bar;
    dsg_partials(u[1], ms, K.md, dn_, dd_);
    ubar[1] = v00_bar * dn_;
    ms_bar += v00_bar * dd_;
    dsg_partials(u[2], ms, K.md, dn_, dd_);
    ubar[2] = v01_bar * dn_;
    ms_bar += v01_bar * dd_;
    dsg_partials(u[4], mf, K.md, dn_, dd_);
    ubar[4] = v10_bar * dn_;
    mf_bar += v10_bar * dd_;
    dsg_partials(u[5], mf, K.md, dn_, dd_);
    ubar[5] = v11_bar * dn_;
    mf_bar += v11_bar * dd_;
    ubar[0] = ms_bar;
    ubar[3] = mf_bar;
}

// Slot of field k of the box cell (a, c) = (i - 1 + c, j - 1 + a), or -1 if
// the source does not read that field there (the inverse of src_slot).
__device__ __forceinline__ int box_slot(int a, int c, int k)
{
    if (a == 1 && c == 1) return k;
    const bool edge = a == 1 || c == 1;
    if (edge) {
        const int n = (a == 1) ? (c == 2 ? 0 : 1) : (a == 2 ? 2 : 3);
        const int f = k == 0 ? 0 : (k >= 3 ? k - 2 : -1);
        return f < 0 ? -1 : 6 + 4 * n + f;
    }
    if (k < 3) return -1;
    const int n = (a == 2 ? 0 : 2) + (c == 2 ? 0 : 1);
    return 22 + 3 * n + (k - 3);
}

// Transpose of one viscous face term (visc_xface_c for d = 0, visc_yface_c
// for d = 1): cotangents (l0, l1) of its two outputs pulled back to its ten
// scalar inputs (u0, w0, u1, w1, cd u0, cd w0, cd u1, cd w1, Jh0, Jh1).  The
// terms are bilinear in the velocity differences and J_b h, so the reverse
// is written out.
template <typename T>
__device__ __forceinline__ void visc_face_vjp(int d, const T in[10], const Geo<T>& ga, const Geo<T>& gb, T h, T l0,
                                              T l1, T lin[10])
{
    const T A11 = T(0.5) * (ga.A11 + gb.A11), A12 = T(0.5) * (ga.A12 + gb.A12);
    const T A21 = T(0.5) * (ga.A21 + gb.A21), A22 = T(0.5) * (ga.A22 + gb.A22);
    const T Jh = T(0.5) * (in[8] + in[9]);
    const T nu = (in[2] - in[0]) / h, nw = (in[3] - in[1]) / h;      // normal differences
    const T tu = T(0.5) * (in[4] + in[6]), tw = T(0.5) * (in[5] + in[7]);  // tangential (mean central)
    T nu_b, nw_b, tu_b, tw_b, Jh_b;
    if (d == 0) {
        // FX = 2 Jh (A11 u_x + A21 u_y), FY = Jh (A12 u_x + A22 u_y + A11 w_x + A21 w_y)
        const T PX = A11 * nu + A21 * tu, PY = A12 * nu + A22 * tu + A11 * nw + A21 * tw;
        Jh_b = l0 * T(2) * PX + l1 * PY;
        nu_b = l0 * T(2) * Jh * A11 + l1 * Jh * A12;
        tu_b = l0 * T(2) * Jh * A21 + l1 * Jh * A22;
        nw_b = l1 * Jh * A11;
        tw_b = l1 * Jh * A21;
    } else {
        // GX = Jh (A12 u_x + A22 u_y + A11 w_x + A21 w_y), GY = 2 Jh (A12 w_x + A22 w_y)
        const T QX = A12 * tu + A22 * nu + A11 * tw + A21 * nw, QY = A12 * tw + A22 * nw;
        Jh_b = l0 * QX + l1 * T(2) * QY;
        tu_b = l0 * Jh * A12;
        nu_b = l0 * Jh * A22;
        tw_b = l0 * Jh * A11 + l1 * T(2) * Jh * A12;
        nw_b = l0 * Jh * A21 + l1 * T(2) * Jh * A22;
    }
    lin[0] = -nu_b / h;
    lin[2] = nu_b / h;
    lin[1] = -nw_b / h;
    lin[3] = nw_b / h;
    lin[4] = lin[6] = T(0.5) * tu_b;
    lin[5] = lin[7] = T(0.5) * tw_b;
    lin[8] = lin[9] = T(0.5) * Jh_b;
}

// Pass B, sources: cotangent dt * GT_c (momentum components) pulled back
// through S_c to its 34 input slots (lam[34]).  Chain rule over the
// structure of cell_sources: the local sources of the cell's six fields and of
// the two fluid-pressure gradients (8 dual evaluations of sources), the
// gradients to the neighbours' thicknesses (fluid_G), and the viscous
// operator through its four face terms, the central differences and the
// desingularised velocities of the 3 x 3 box.
template <typename T>
__device__ __forceinline__ void adj_src_lam(const KParams& P, const T* __restrict__ U, const T* __restrict__ GT,
                                            const T* __restrict__ b, T dt, int i, int j, T lam[34])
{
    const size_t c = (size_t)j * P.pitch + i, fs = (size_t)P.ny * P.pitch;
    Stencil<T> s;
    load_stencil(P, U, i, j, s);
    const Geo5<T> g5 = geo5(P, b, i, j);
    T gS[NF];
    for (int k = 0; k < NF; k++) gS[k] = dt * GT[k * fs + c];
    using TT = Dual<T>;
    const Consts<TT> K(P);
    const Geo<TT> gW = lift(g5.W), gE = lift(g5.E), gSo = lift(g5.S), gN = lift(g5.N);
    for (int q = 0; q < 34; q++) lam[q] = T(0);
    const T two_dxi = T(P.two_dxi), two_deta = T(P.two_deta);
    TT dn[6];
    dn[0] = TT((g5.E.nX - g5.W.nX) / two_dxi, T(0));
    dn[1] = TT((g5.E.nY - g5.W.nY) / two_dxi, T(0));
    dn[2] = TT((g5.E.nZ - g5.W.nZ) / two_dxi, T(0));
    dn[3] = TT((g5.N.nX - g5.S.nX) / two_deta, T(0));
    dn[4] = TT((g5.N.nY - g5.S.nY) / two_deta, T(0));
    dn[5] = TT((g5.N.nZ - g5.S.nZ) / two_deta, T(0));
    auto fg = [&](const T* u, const Geo<TT>& g, int dir) {
        return fluid_G(TT(u[0], dir == 0 ? T(1) : T(0)), TT(u[3], dir == 1 ? T(1) : T(0)), g);
    };
    const T dGx = ((fg(s.row[3], gE, -1) - fg(s.row[1], gW, -1)) / K.two_dxi).v;
    const T dGy = ((fg(s.col[3], gN, -1) - fg(s.col[1], gSo, -1)) / K.two_deta).v;

    // viscous operator: values of the box velocities, thickness products,
    // central differences and face terms
    T u9[3][3], w9[3][3], Jh[5], cyu[3], cyw[3], cxu[3], cxw[3], SvX = T(0), SvY = T(0);
    const Consts<T> Kb(P);
    if (P.visc) {
        for (int a = 0; a < 3; a++)
            for (int cc = 0; cc < 3; cc++) {
                u9[a][cc] = dsg(s.box[a][cc][4], s.box[a][cc][3], Kb.md);
                w9[a][cc] = dsg(s.box[a][cc][5], s.box[a][cc][3], Kb.md);
            }
        Jh[0] = s.row[2][0] + s.row[2][3];  // C
        Jh[1] = s.row[1][0] + s.row[1][3];  // W
        Jh[2] = s.row[3][0] + s.row[3][3];  // E
        Jh[3] = s.col[1][0] + s.col[1][3];  // S
        Jh[4] = s.col[3][0] + s.col[3][3];  // N
        for (int q = 0; q < 3; q++) {
            cyu[q] = cdiff(u9[2][q], u9[0][q], Kb.deta);
            cyw[q] = cdiff(w9[2][q], w9[0][q], Kb.deta);
            cxu[q] = cdiff(u9[q][2], u9[q][0], Kb.dxi);
            cxw[q] = cdiff(w9[q][2], w9[q][0], Kb.dxi);
        }
        T FX0, FY0, FX1, FY1, GX0, GY0, GX1, GY1;
        visc_xface_c(u9[1][0], w9[1][0], u9[1][1], w9[1][1], cyu[0], cyw[0], cyu[1], cyw[1], Jh[1], Jh[0], g5.W, g5.C,
                     Kb.dxi, FX0, FY0);
        visc_xface_c(u9[1][1], w9[1][1], u9[1][2], w9[1][2], cyu[1], cyw[1], cyu[2], cyw[2], Jh[0], Jh[2], g5.C, g5.E,
                     Kb.dxi, FX1, FY1);
        visc_yface_c(u9[0][1], w9[0][1], u9[1][1], w9[1][1], cxu[0], cxw[0], cxu[1], cxw[1], Jh[3], Jh[0], g5.S, g5.C,
                     Kb.deta, GX0, GY0);
        visc_yface_c(u9[1][1], w9[1][1], u9[2][1], w9[2][1], cxu[1], cxw[1], cxu[2], cxw[2], Jh[0], Jh[4], g5.C, g5.N,
                     Kb.deta, GX1, GY1);
        SvX = (FX1 - FX0) / Kb.dxi + (GX1 - GX0) / Kb.deta;
        SvY = (FY1 - FY0) / Kb.dxi + (GY1 - GY0) / Kb.deta;
    }

    // (1) local sources: the cell's six fields and the two gradients, by the
    // reverse sweep of sources() (the viscous prefactor eps phi^f / N_R enters
    // through phi^f)
    T lGx = T(0), lGy = T(0);
    {
        const Consts<T> Kl(P);
        T L[2][2] = {{gS[1], gS[2]}, {gS[4], gS[5]}};
        T Lphif = T(0);
        if (P.visc) Lphif = Kl.eps * Kl.inv_n_r * (gS[4] * SvX + gS[5] * SvY);
        T dn_b[6];
        for (int q = 0; q < 6; q++) dn_b[q] = dn[q].v;
        T ub[NF];
        sources_vjp(Kl, P.flags, s.row[2], g5.C, dn_b, dGx, dGy, L, Lphif, ub, lGx, lGy);
        for (int k = 0; k < NF; k++) lam[k] += ub[k];
    }
    // (2) gradients of J_b h pbar^f to the neighbours' m^s, m^f
    {
        const T* cell[4] = {s.row[3], s.row[1], s.col[3], s.col[1]};  // E, W, N, S
        const Geo<TT>* geo[4] = {&gE, &gW, &gN, &gSo};
        const T coef[4] = {lGx, -lGx, lGy, -lGy};
        for (int n = 0; n < 4; n++) {
            const TT den = n < 2 ? K.two_dxi : K.two_deta;
            for (int dir = 0; dir < 2; dir++) lam[6 + 4 * n + dir] += coef[n] * (fg(cell[n], *geo[n], dir) / den).d;
        }
    }
    // (3) viscous operator
    if (P.visc) {
        const T phif = dsg(s.row[2][3], s.row[2][0] + s.row[2][3], Kb.md);
        const T coef = Kb.eps * phif * Kb.inv_n_r;
        const T lX = gS[4] * coef, lY = gS[5] * coef;
        T lu9[3][3], lw9[3][3], lJh[5], lcyu[3], lcyw[3], lcxu[3], lcxw[3];
        for (int a = 0; a < 3; a++)
            for (int cc = 0; cc < 3; cc++) lu9[a][cc] = lw9[a][cc] = T(0);
        for (int q = 0; q < 5; q++) lJh[q] = T(0);
        for (int q = 0; q < 3; q++) lcyu[q] = lcyw[q] = lcxu[q] = lcxw[q] = T(0);
        T in[10], lin[10];
        // x-face i - 1/2 (FX0, FY0) enters with -1/dxi, x-face i + 1/2 with +1/dxi
        for (int f = 0; f < 2; f++) {
            const int c0 = f, c1 = f + 1;
            in[0] = u9[1][c0];
            in[1] = w9[1][c0];
            in[2] = u9[1][c1];
            in[3] = w9[1][c1];
            in[4] = cyu[c0];
            in[5] = cyw[c0];
            in[6] = cyu[c1];
            in[7] = cyw[c1];
            in[8] = f == 0 ? Jh[1] : Jh[0];
            in[9] = f == 0 ? Jh[0] : Jh[2];
            const T sg = f == 0 ? T(-1) : T(1);
            visc_face_vjp(0, in, f == 0 ? g5.W : g5.C, f == 0 ? g5.C : g5.E, Kb.dxi, sg * lX / Kb.dxi,
                          sg * lY / Kb.dxi, lin);
            lu9[1][c0] += lin[0];
            lw9[1][c0] += lin[1];
            lu9[1][c1] += lin[2];
            lw9[1][c1] += lin[3];
            lcyu[c0] += lin[4];
            lcyw[c0] += lin[5];
            lcyu[c1] += lin[6];
            lcyw[c1] += lin[7];
            lJh[f == 0 ? 1 : 0] += lin[8];
            lJh[f == 0 ? 0 : 2] += lin[9];
        }
        // y-face j - 1/2 (GX0, GY0) with -1/deta, y-face j + 1/2 with +1/deta
        for (int f = 0; f < 2; f++) {
            const int a0 = f, a1 = f + 1;
            in[0] = u9[a0][1];
            in[1] = w9[a0][1];
            in[2] = u9[a1][1];
            in[3] = w9[a1][1];
            in[4] = cxu[a0];
            in[5] = cxw[a0];
            in[6] = cxu[a1];
            in[7] = cxw[a1];
            in[8] = f == 0 ? Jh[3] : Jh[0];
            in[9] = f == 0 ? Jh[0] : Jh[4];
            const T sg = f == 0 ? T(-1) : T(1);
            visc_face_vjp(1, in, f == 0 ? g5.S : g5.C, f == 0 ? g5.C : g5.N, Kb.deta, sg * lX / Kb.deta,
                          sg * lY / Kb.deta, lin);
            lu9[a0][1] += lin[0];
            lw9[a0][1] += lin[1];
            lu9[a1][1] += lin[2];
            lw9[a1][1] += lin[3];
            lcxu[a0] += lin[4];
            lcxw[a0] += lin[5];
            lcxu[a1] += lin[6];
            lcxw[a1] += lin[7];
            lJh[f == 0 ? 3 : 0] += lin[8];
            lJh[f == 0 ? 0 : 4] += lin[9];
        }
        // central differences (up - dn) / (2 h)
        for (int q = 0; q < 3; q++) {
            const T ry = lcyu[q] / (T(2) * Kb.deta), rw = lcyw[q] / (T(2) * Kb.deta);
            lu9[2][q] += ry;
            lu9[0][q] -= ry;
            lw9[2][q] += rw;
            lw9[0][q] -= rw;
            const T rx = lcxu[q] / (T(2) * Kb.dxi), rxw = lcxw[q] / (T(2) * Kb.dxi);
            lu9[q][2] += rx;
            lu9[q][0] -= rx;
            lw9[q][2] += rxw;
            lw9[q][0] -= rxw;
        }
        // desingularised velocities u = dsg(p^f_X, m^f), w = dsg(p^f_Y, m^f)
        for (int a = 0; a < 3; a++)
            for (int cc = 0; cc < 3; cc++) {
                const T* bx = s.box[a][cc];
                const TT dup = dsg(TT(bx[4], T(1)), TT(bx[3], T(0)), K.md);
                const TT dum = dsg(TT(bx[4], T(0)), TT(bx[3], T(1)), K.md);
                const TT dwp = dsg(TT(bx[5], T(1)), TT(bx[3], T(0)), K.md);
                const TT dwm = dsg(TT(bx[5], T(0)), TT(bx[3], T(1)), K.md);
                lam[box_slot(a, cc, 4)] += lu9[a][cc] * dup.d;
                lam[box_slot(a, cc, 5)] += lw9[a][cc] * dwp.d;
                lam[box_slot(a, cc, 3)] += lu9[a][cc] * dum.d + lw9[a][cc] * dwm.d;
            }
        // J_b h = m^s + m^f of C, W, E, S, N
        const int ba[5] = {1, 1, 1, 0, 2}, bc[5] = {1, 0, 2, 1, 1};
        for (int q = 0; q < 5; q++) {
            lam[box_slot(ba[q], bc[q], 0)] += lJh[q];
            lam[box_slot(ba[q], bc[q], 3)] += lJh[q];
        }
    }
}

// Wavefronts of sources per grid row: each covers 60 target columns of the
// row extended by one ghost column per side (extended column t + 1).
__host__ __device__ inline int adj_swaves(int nx) { return (nx + 2 + 59) / 60; }

// Pass B, sources, per grid row of source cells: lane l of wavefront w takes
// source cell c = 60 w - 2 + l (cells outside the grid contribute zeros) and
// lanes 1..60 sum, for target column t = c (fixed order: own, west neighbour's,
// east neighbour's slots), what lands on (t, j) [6 fields], on (t, j + 1)
// and on (t, j - 1) [fields 0, 3, 4, 5 each] into SS[14][ny][nx + 2] at
// extended column t + 1 (source row j), ghost columns included.
template <typename T>
__global__ void __launch_bounds__(128) k_adj_src(KParams P, const T* __restrict__ U, const T* __restrict__ GT,
                                                 const T* __restrict__ b, T dt, T* __restrict__ SS)
{
    const int j = (int)blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int w = (int)blockIdx.x * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6);
    if (w >= adj_swaves(P.nx)) return;  // whole wavefront
    const int c = 60 * w - 2 + lane;
    T lam[34];
    if (c >= 0 && c < P.nx)
        adj_src_lam(P, U, GT, b, dt, c, j, lam);
    else
        for (int q = 0; q < 34; q++) lam[q] = T(0);
    // every lane of the wavefront takes part in the shuffles.  Slots: 0..5
    // centre; 6 + 4 n + f neighbour n (E, W, N, S) field (0, 3, 4, 5)[f];
    // 22 + 3 n + f corner n (NE, NW, SE, SW) field 3 + f.
    T o[14];
#pragma unroll
    for (int k = 0; k < NF; k++) o[k] = lam[k];
#pragma unroll
    for (int f = 0; f < 4; f++) {
        const int k = f == 0 ? 0 : 2 + f;  // field 0, 3, 4, 5
        o[k] = (o[k] + __shfl(lam[6 + f], lane - 1, 64)) + __shfl(lam[10 + f], lane + 1, 64);
        T up = lam[14 + f], dn = lam[18 + f];
        if (f > 0) {
            up = (up + __shfl(lam[22 + f - 1], lane - 1, 64)) + __shfl(lam[25 + f - 1], lane + 1, 64);
            dn = (dn + __shfl(lam[28 + f - 1], lane - 1, 64)) + __shfl(lam[31 + f - 1], lane + 1, 64);
        }
        o[6 + f] = up;
        o[10 + f] = dn;
    }
    const int e = c + 1;
    if (lane >= 1 && lane <= 60 && e < P.nx + 2) {
        const size_t nss = (size_t)P.ny * (P.nx + 2), off = (size_t)j * (P.nx + 2) + e;
#pragma unroll
        for (int q = 0; q < 14; q++) SS[q * nss + off] = o[q];
    }
}

// Pass C: lam_in(k) = DU(k) + all face and source contributions that land on
// cell k through the ghost map, summed in a fixed order.  Cells two or more
// away from every edge take the direct path below (no ghost cell maps onto
// them); the ring of edge cells walks the ghost map (k_adj_gather).  With z
// given, lam_in = (DU + contributions) + zc z (z may be lam_in itself: each
// cell reads its own z before writing).
template <typename T>
__device__ __forceinline__ void adj_gather_interior(const KParams& P, const T* __restrict__ DU,
                                                    const T* __restrict__ XS, const T* __restrict__ FCY,
                                                    const T* __restrict__ SS, const T* z, T zc, T* lam_in, int i,
                                                    int j)
{
    const size_t c = (size_t)j * P.pitch + i, fs = (size_t)P.ny * P.pitch;
    // slot-major cotangent arrays (slot stride: number of faces or cells)
    const size_t nxs = (size_t)P.ny * (P.nx + 4), nfy = (size_t)P.nx * (P.ny + 1), nss = (size_t)P.ny * (P.nx + 2);
    T acc[NF];
    for (int k = 0; k < NF; k++) acc[k] = DU[k * fs + c];
    // No ghost cell maps onto this cell: each contribution comes from a
    // fixed (face or cell, slot); x-faces (summed per cell), y-faces, then
    // the 3 x 3 sources.
    {
        const T* f = XS + (size_t)j * (P.nx + 4) + (i + 2);
        for (int k = 0; k < NF; k++) acc[k] += f[k * nxs];
    }
    for (int fj = j - 2; fj <= j + 1; fj++) {
        const T* f = FCY + ((size_t)(fj + 1) * P.nx + i) + 6 * (j - fj + 1) * nfy;
        for (int k = 0; k < NF; k++) acc[k] += f[k * nfy];
    }
    // sources: what lands on this cell from source rows j, j - 1 (upward) and
    // j + 1 (downward), each already summed over the three source columns
    {
        const size_t o = (size_t)(i + 1);
        const T* f0 = SS + (size_t)j * (P.nx + 2) + o;
        const T* fu = SS + (size_t)(j - 1) * (P.nx + 2) + o;
        const T* fd = SS + (size_t)(j + 1) * (P.nx + 2) + o;
        for (int k = 0; k < NF; k++) acc[k] += f0[k * nss];
        const int kk[4] = {0, 3, 4, 5};
        for (int f = 0; f < 4; f++) acc[kk[f]] += fu[(6 + f) * nss];
        for (int f = 0; f < 4; f++) acc[kk[f]] += fd[(10 + f) * nss];
    }
    for (int k = 0; k < NF; k++) lam_in[k * fs + c] = z ? acc[k] + zc * z[k * fs + c] : acc[k];
}

// Edge ring: the cells outside the interior box, enumerated as the bottom
// two rows, the top two rows, then the two first and two last columns of the
// rows between (every cell when the grid is narrower than five cells).
__host__ __device__ inline long long adj_ring_cells(int nx, int ny)
{
    const int nbot = ny < 2 ? ny : 2, ntop = (ny - nbot) < 2 ? (ny - nbot) : 2, mid = ny - nbot - ntop;
    const int ncol = nx <= 4 ? nx : 4;
    return (long long)(nbot + ntop) * nx + (long long)mid * ncol;
}

// Pass C in one launch of 128-thread workgroups (the two kinds of cell get
// separate workgroups, so no wavefront mixes the paths).  Workgroups 0 .. nbi-1
// cover the interior box i in [2, nx - 3], j in [2, ny - 3] (nbx workgroups of
// 128 cells per row), one thread per cell.  The rest cover the edge ring with
// one wavefront per ring cell: the lanes share the candidate contributions
// (the cell's own and the four ghost columns' x-face sums, 24 y-face (face,
// stencil position) pairs, and the source sums landing on the 3 x 3 targets
// (cell or ghost, from the source row below, level or above)), keep those the
// ghost map sends to this cell, and the lanes' partial sums are combined by a fixed
// butterfly (deterministic).
template <typename T>
__global__ void __launch_bounds__(128) k_adj_gather(KParams P, const T* __restrict__ DU, const T* __restrict__ XS,
                                                    const T* __restrict__ FCY, const T* __restrict__ SS, const T* z,
                                                    T zc, T* lam_in, int nbi, int nbx)
{
    if ((int)blockIdx.x < nbi) {
        const int i = 2 + ((int)blockIdx.x % nbx) * 128 + (int)threadIdx.x;
        const int j = 2 + (int)blockIdx.x / nbx;
        if (i <= P.nx - 3) adj_gather_interior(P, DU, XS, FCY, SS, z, zc, lam_in, i, j);
        return;
    }
    const long long r = ((long long)(blockIdx.x - nbi) * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    const int nx = P.nx, ny = P.ny;
    if (r >= adj_ring_cells(nx, ny)) return;  // whole wavefront
    const int nbot = ny < 2 ? ny : 2, ntop = (ny - nbot) < 2 ? (ny - nbot) : 2;
    const int ncol = nx <= 4 ? nx : 4;
    int i, j;
    if (r < (long long)nbot * nx) {
        j = (int)(r / nx);
        i = (int)(r % nx);
    } else if (r < (long long)(nbot + ntop) * nx) {
        const long long r2 = r - (long long)nbot * nx;
        j = ny - ntop + (int)(r2 / nx);
        i = (int)(r2 % nx);
    } else {
        const long long r3 = r - (long long)(nbot + ntop) * nx;
        j = nbot + (int)(r3 / ncol);
        const int cc = (int)(r3 % ncol);
        i = nx <= 4 ? cc : (cc < 2 ? cc : nx - 4 + cc);
    }
    const size_t fs = (size_t)ny * P.pitch;
    const size_t nxs = (size_t)ny * (nx + 4), nfy = (size_t)nx * (ny + 1), nss = (size_t)ny * (nx + 2);
    T acc[NF];
#pragma unroll
    for (int k = 0; k < NF; k++) acc[k] = T(0);
    for (int it = lane; it < 5 + 24 + 27; it += 64) {
        if (it < 5) {
            // x-face sums: this cell's, then the ghost columns -2, -1, nx, nx+1
            // when the ghost map sends them here (normal momenta flip at walls)
            const int g = it == 0 ? i : (it == 1 ? -2 : (it == 2 ? -1 : nx + it - 3));
            int flip = 0;
            if (it > 0 && map_index(g, nx, P.bc[0], P.bc[1], flip) != i) continue;
            const T* f = XS + (size_t)j * (nx + 4) + (g + 2);
#pragma unroll
            for (int k = 0; k < NF; k++) {
                const T v = f[k * nxs];
                acc[k] += (flip && (k == 1 || k == 4)) ? -v : v;
            }
        } else if (it < 29) {
            // y-face fj within 3 rows, stencil position q
            const int fo = (it - 5) / 4, q = (it - 5) % 4;
            const int fl = j - 3 + fo;  // face between rows fl and fl + 1
            if (fl < -1 || fl > ny - 1) continue;
            int flip = 0;
            if (map_index(fl - 1 + q, ny, P.bc[2], P.bc[3], flip) != j) continue;
            const T* f = FCY + ((size_t)(fl + 1) * nx + i);
#pragma unroll
            for (int k = 0; k < NF; k++) {
                const T v = f[(6 * q + k) * nfy];
                acc[k] += (flip && (k == 2 || k == 5)) ? -v : v;
            }
        } else {
            // target (ti, tj) in {i, ghost columns} x {j, ghost rows} of the
            // source sums: level (source row tj), upward (tj - 1), downward (tj + 1)
            const int s2 = it - 29, kind = s2 / 9, ti_c = (s2 % 9) % 3, tj_c = (s2 % 9) / 3;
            const int ti = ti_c == 0 ? i : (ti_c == 1 ? -1 : nx), tj = tj_c == 0 ? j : (tj_c == 1 ? -1 : ny);
            int fx = 0, fy = 0;
            if (map_index(ti, nx, P.bc[0], P.bc[1], fx) != i || map_index(tj, ny, P.bc[2], P.bc[3], fy) != j) continue;
            if (ti_c != 0 && ti == i) continue;  // a ghost column never equals the cell
            const int sr = kind == 0 ? tj : (kind == 1 ? tj - 1 : tj + 1);  // source row
            if (sr < 0 || sr >= ny) continue;
            const T* f = SS + (size_t)sr * (nx + 2) + (ti + 1);
            if (kind == 0) {
#pragma unroll
                for (int k = 0; k < NF; k++) {
                    T v = f[k * nss];
                    if (fx && (k == 1 || k == 4)) v = -v;
                    if (fy && (k == 2 || k == 5)) v = -v;
                    acc[k] += v;
                }
            } else {
                const int base = kind == 1 ? 6 : 10;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const int k = q == 0 ? 0 : 2 + q;
                    T v = f[(base + q) * nss];
                    if (fx && k == 4) v = -v;
                    if (fy && k == 5) v = -v;
                    acc[k] += v;
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NF; k++)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) acc[k] += __shfl_xor(acc[k], off, 64);
    if (lane < NF) {
        T v = acc[0];
#pragma unroll
        for (int k = 1; k < NF; k++) v = lane == k ? acc[k] : v;
        const size_t c = (size_t)j * P.pitch + i;
        const T o = DU[lane * fs + c] + v;
        lam_in[lane * fs + c] = z ? o + zc * z[lane * fs + c] : o;
    }
}

// Loss 1/2 sum (h - h_target)^2 dx dy (h bed-normal, m) and, if lam is not
// null, its cotangent with respect to the state (m^s and m^f entries); FP64
// partial sums per block.
template <typename T>
__global__ void __launch_bounds__(256) k_loss(KParams P, const T* __restrict__ U, const T* __restrict__ b,
                                              const double* __restrict__ target, T* __restrict__ lam,
                                              double* __restrict__ part)
{
    __shared__ double sh[256];
    const int tid = threadIdx.x;
    const size_t n = (size_t)P.nx * P.ny, fs = (size_t)P.ny * P.pitch;
    double acc = 0.0;
    for (size_t q = (size_t)blockIdx.x * 256 + tid; q < n; q += (size_t)gridDim.x * 256) {
        const int j = (int)(q / P.nx), i = (int)(q - (size_t)j * P.nx);
        const size_t c = (size_t)j * P.pitch + i;
        auto bv = [&](int ii, int jj) { return (double)b[(size_t)(jj + BHALO) * P.bpitch + BOFF + ii]; };
        const Geo<double> g = geometry(bv(i + 1, j), bv(i - 1, j), bv(i, j + 1), bv(i, j - 1), P.two_dxi, P.two_deta);
        const double h = ((double)U[c] + (double)U[3 * fs + c]) / g.J * P.H;
        const double r = h - target[q];
        acc += 0.5 * r * r * P.dx * P.dy;
        if (lam) {  // the loss alone is asked for without it
            const double gm = r * P.dx * P.dy * P.H / g.J;
            for (int k = 0; k < NF; k++) lam[k * fs + c] = T(0);
            lam[c] = T(gm);
            lam[3 * fs + c] = T(gm);
        }
    }
    sh[tid] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    if (tid == 0) part[blockIdx.x] = sh[0];
}

// FP64 partial dot products of two [6][ny][pitch] arrays.
template <typename T>
__global__ void __launch_bounds__(256) k_dot(KParams P, const T* __restrict__ x, const T* __restrict__ y,
                                             double* __restrict__ part)
{
    __shared__ double sh[256];
    const int tid = threadIdx.x;
    const size_t n = (size_t)P.nx * P.ny, fs = (size_t)P.ny * P.pitch;
    double acc = 0.0;
    for (size_t q = (size_t)blockIdx.x * 256 + tid; q < n; q += (size_t)gridDim.x * 256) {
        const int j = (int)(q / P.nx), i = (int)(q - (size_t)j * P.nx);
        const size_t c = (size_t)j * P.pitch + i;
        for (int k = 0; k < NF; k++) acc += (double)x[k * fs + c] * (double)y[k * fs + c];
    }
    sh[tid] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    if (tid == 0) part[blockIdx.x] = sh[0];
}

}  // namespace m2p
