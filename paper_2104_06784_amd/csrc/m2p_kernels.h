// m2p_kernels.h -- HIP kernels of the step: stage kernels (forward-Euler
// stage of Sect. 2.2's scheme, fused reconstruction + fluxes + sources +
// update), the per-step finalize (time, CFL dt, boundary integrals, inflow
// states), and state conversion / reduction kernels.  Included once per
// precision by m2p_f64.hip and m2p_f32.hip.
#pragma once

#include "m2p_device.h"
#include "m2p_launch.h"

namespace m2p {

// ---------------------------------------------------------------- helpers

// Mode-II state segment covering boundary index k of a side, or -1
__device__ __forceinline__ int state_seg_at(const KParams& P, int side, int k)
{
    for (int s = 0; s < P.nsseg; s++)
        if (P.sseg[s].side == side && k >= P.sseg[s].i0 && k < P.sseg[s].i0 + P.sseg[s].ncells) return s;
    return -1;
}

// Ghost cell (ii, jj) outside exactly one side and next to a Mode-II state
// segment takes that segment's prescribed inflowing state (gh: the stage's
// ghost states); other ghost cells keep the boundary rule's value.
template <typename T>
__device__ __forceinline__ void ghost_sub(const KParams& P, const double (*gh)[NF], int ii, int jj, T u[NF])
{
    int side = -1, k = 0;
    if (jj < 0) {
        side = 2;
        k = ii;
    } else if (jj >= P.ny) {
        side = 3;
        k = ii;
    } else if (ii < 0) {
        side = 0;
        k = jj;
    } else if (ii >= P.nx) {
        side = 1;
        k = jj;
    }
    if (side < 0 || k < 0 || k >= (side < 2 ? P.ny : P.nx)) return;
    const int s = state_seg_at(P, side, k);
    if (s < 0) return;
#pragma unroll
    for (int f = 0; f < NF; f++) u[f] = T(gh[s][f]);
}

template <typename T>
struct View {
    const KParams& P;
    const T* U;
    const T* b;
    size_t fs;
    const double (*gh)[NF];  // ghost states of Mode-II state segments (stage kernels), else null
    __device__ View(const KParams& P_, const T* U_, const T* b_, const double (*gh_)[NF] = nullptr)
        : P(P_), U(U_), b(b_), fs((size_t)P_.ny * P_.pitch), gh(gh_) {}
    // state at any (ii, jj) in [-2, n+1] with the boundary rules applied
    __device__ __forceinline__ void load(int ii, int jj, T u[NF]) const
    {
        int fx = 0, fy = 0;
        int mi = map_index(ii, P.nx, P.bc[0], P.bc[1], fx);
        int mj = map_index(jj, P.ny, P.bc[2], P.bc[3], fy);
        size_t c = (size_t)mj * P.pitch + mi;
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
        if (gh && P.nsseg > 0) ghost_sub(P, gh, ii, jj, u);
    }
    __device__ __forceinline__ T bv(int ii, int jj) const { return b[(size_t)(jj + BHALO) * P.bpitch + BOFF + ii]; }
    __device__ __forceinline__ Geo<T> geo(int ii, int jj, const Consts<T>& K) const
    {
        return geometry(bv(ii + 1, jj), bv(ii - 1, jj), bv(ii, jj + 1), bv(ii, jj - 1), K.two_dxi, K.two_deta);
    }
};

// inflow segment covering boundary index k of a side, or -1
__device__ __forceinline__ int inflow_seg_at(const KParams& P, int side, int k)
{
    for (int s = 0; s < P.nseg; s++)
        if (P.seg[s].side == side && k >= P.seg[s].i0 && k < P.seg[s].i0 + P.seg[s].ncells) return s;
    return -1;
}

template <typename T>
__device__ __forceinline__ void reconstruct(const T w[4][NF], T uL[NF], T uR[NF])
{
    // cells (a-1, a, a+1, a+2) -> face a+1/2
#pragma unroll
    for (int k = 0; k < NF; k++) {
        T wm = w[0][k], w0 = w[1][k], w1 = w[2][k], w2 = w[3][k];
        T s0 = minmod(w0 - wm, w1 - w0);
        T s1 = minmod(w1 - w0, w2 - w1);
        uL[k] = w0 + T(0.5) * s0;
        uR[k] = w1 - T(0.5) * s1;
    }
}

// Deterministic block reduction (fixed tree) of NV doubles; result in lane 0 of thread 0.
template <int NV, int NT>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh)
{
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
#pragma unroll
    for (int q = 0; q < NV; q++) sh[q * NT + tid] = v[q];
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (tid < s)
#pragma unroll
            for (int q = 0; q < NV; q++) sh[q * NT + tid] += sh[q * NT + tid + s];
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NV; q++) v[q] = sh[q * NT];
}

// Outflow through one boundary face in one stage: f0, f1 = the sign-adjusted
// volume flux of each phase times the face length, stored in the stage's slot
// of bpart ([kOutSlots][4][nmax][2]: slot 0 holds the running integrals, slot
// 1 + s stage slot s; then the step's dt at outflow_dt_index).  The finalize
// adds the weighted slots to the integrals (a read-modify-write of the
// integral here would keep its address, value and weight live across the
// march).
__device__ __forceinline__ void put_outflow(double* __restrict__ bpart, int nmax, int slot, int side, int k,
                                            double f0, double f1)
{
    double* v = bpart + ((size_t)((1 + slot) * 4 + side) * nmax + k) * 2;
    v[0] = f0;
    v[1] = f1;
}

// quadrature weight of stage slot s (the stage kinds of stage_slot, in order)
__device__ __forceinline__ double slot_weight(int s, int rk)
{
    return stage_weight(s == 0 ? 1 : (rk == 2 ? 2 : (s == 1 ? 3 : 4)), rk);
}

// Boundary face q ([4][nmax], side-major): the step's stage fluxes, each
// times its weight times dt, added to the face's running integral in stage
// order.
__device__ __forceinline__ void outflow_accumulate(const KParams& P, double* __restrict__ bpart, int nmax, int q)
{
    const int side = q / nmax, k = q - side * nmax;
    if (side >= 4 || k >= (side < 2 ? P.ny : P.nx)) return;
    const double dt = bpart[outflow_dt_index(nmax)];
    double* acc = bpart + (size_t)q * 2;
    const size_t slot = (size_t)4 * nmax * 2;
    double a0 = acc[0], a1 = acc[1];
    for (int s = 0; s < P.rk; s++) {
        const double w = slot_weight(s, P.rk) * dt;
        a0 += w * acc[(s + 1) * slot];
        a1 += w * acc[(s + 1) * slot + 1];
    }
    acc[0] = a0;
    acc[1] = a1;
}

// -------------------------------------------------- reference stage kernel

// One thread per cell; every stencil value is read from memory.  STAGE is
// the stage kind (stage_combine): kind 1 writes E(U^n) at t^n; kinds 2-4
// combine E(Uin) with the cell's own U^n (read from Un) and write Uout
// (kinds 2 and 4 over U^n, with the maximum phase speeds of the new state
// for the next CFL step).
template <typename T, int STAGE, bool WB = false>
__global__ void __launch_bounds__(256) k_stage_ref(KParams P, const T* __restrict__ Uin, T* Un, T* Uout,
                                                   const T* __restrict__ b, const T* __restrict__ mu,
                                                   DevScalars* __restrict__ S, double* __restrict__ bpart,
                                                   double* __restrict__ wpart, int nmax,
                                                   const T* __restrict__ KE)
{
    __shared__ double sh[9 * 256];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const Consts<T> K(P);
    const View<T> V(P, Uin, b, S->sghost[stage_slot(STAGE)]);
    const bool active = i < P.nx && j < P.ny;
    double red[1] = {0};  // clamps
    double ax = 0.0, ay = 0.0;
    int bad = 0;
    // earth-pressure coefficient of cell (ii, jj) in direction d (a ghost
    // cell: that of the cell it maps to); 1 without the option
    const bool ep = (P.flags & kFlagEarthPressure) != 0;
    const size_t kfs = (size_t)P.ny * P.pitch;
    auto kep = [&](int ii, int jj, int d) {
        if (!ep) return T(1);
        int f = 0;
        const int mi = map_index(ii, P.nx, P.bc[0], P.bc[1], f);
        const int mj = map_index(jj, P.ny, P.bc[2], P.bc[3], f);
        return KE[d * kfs + (size_t)mj * P.pitch + mi];
    };
    if (active) {
        const T dt = T(S->dt);
        T row[5][NF], col[5][NF];
        for (int q = 0; q < 5; q++) V.load(i - 2 + q, j, row[q]);
        for (int q = 0; q < 5; q++) V.load(i, j - 2 + q, col[q]);
        const Geo<T> gC = V.geo(i, j, K), gW = V.geo(i - 1, j, K), gE = V.geo(i + 1, j, K);
        const Geo<T> gS = V.geo(i, j - 1, K), gN = V.geo(i, j + 1, K);
        T HXl[NF], HXr[NF], HYb[NF], HYt[NF], uL[NF], uR[NF];
        // well-balanced option: per direction the cell's pressure corrections
        // and, per phase, its balanced basal-pressure source term
        T cxw[NF], cyw[NF], wbs[4];
        if constexpr (WB) {
            T w[4][NF];
            for (int d = 0; d < 2; d++) {
                const T(*cs)[NF] = d == 0 ? row : col;
                const int n = d == 0 ? P.nx : P.ny, p = d == 0 ? i : j;
                // c^2 of the five cells (a cell two outside the domain takes
                // the c of the ghost cell next to the edge) and their beds
                T c2[5], bb[5];
                for (int q = 0; q < 5; q++) {
                    int pq = p - 2 + q;
                    pq = pq < -1 ? -1 : (pq > n ? n : pq);
                    const T c = d == 0 ? V.geo(pq, j, K).c : V.geo(i, pq, K).c;
                    c2[q] = c * c;
                    bb[q] = d == 0 ? V.bv(i - 2 + q, j) : V.bv(i, j - 2 + q);
                }
                // face values (and bed slopes) of the cells p - 1, p, p + 1
                T em[3][2], ep[3][2], bm[3][2], bp[3][2], sb[3];
                for (int ph = 0; ph < 2; ph++) {
                    T e[5];
                    for (int q = 0; q < 5; q++) e[q] = K.eps * c2[q] * cs[q][3 * ph];
                    for (int q = 1; q < 4; q++)
                        wb_cell(e[q - 1], e[q], e[q + 1], bb[q - 1], bb[q], bb[q + 1], em[q - 1][ph],
                                ep[q - 1][ph], bm[q - 1][ph], bp[q - 1][ph], &sb[q - 1]);
                }
                const Geo<T>& gM = d == 0 ? gW : gS;
                const Geo<T>& gP = d == 0 ? gE : gN;
                // wall faces (not where a state-inflow segment holds the ghost cells)
                const int kb = d == 0 ? j : i;
                const bool lo = P.bc[2 * d] == 1 && state_seg_at(P, 2 * d, kb) < 0;
                const bool hi = P.bc[2 * d + 1] == 1 && state_seg_at(P, 2 * d + 1, kb) < 0;
                T Hm[NF], Hp[NF], cl[NF], cr[NF], cm[NF];
                for (int q = 0; q < 4; q++)
                    for (int k = 0; k < NF; k++) w[q][k] = cs[q][k];
                reconstruct(w, uL, uR);
                wb_face(K, P.flags, uL, gM, c2[1], uR, gC, c2[2], ep[0], bp[0], em[1], bm[1],
                        wb_bed_jump(bb[1], bb[2], sb[0], sb[1]), p == 0 && lo, false, d, Hm, cl, cm);
                for (int q = 0; q < 4; q++)
                    for (int k = 0; k < NF; k++) w[q][k] = cs[q + 1][k];
                reconstruct(w, uL, uR);
                wb_face(K, P.flags, uL, gC, c2[2], uR, gP, c2[3], ep[1], bp[1], em[2], bm[2],
                        wb_bed_jump(bb[2], bb[3], sb[1], sb[2]), false, p + 1 == n && hi, d, Hp, cl, cr);
                T* cw = d == 0 ? cxw : cyw;
                for (int k = 0; k < NF; k++) {
                    cw[k] = cl[k] - cm[k];
                    (d == 0 ? HXl : HYb)[k] = Hm[k];
                    (d == 0 ? HXr : HYt)[k] = Hp[k];
                }
                for (int ph = 0; ph < 2; ph++) {
                    const T fac = ph == 0 ? T(1) - K.al : T(1);
                    // (the FP32 forms take the bed slope itself for the face difference)
                    const T db = Folded<T>::value ? sb[1] : bp[1][ph] - bm[1][ph];
                    wbs[2 * ph + d] =
                        -(fac / K.eps) * (T(0.5) * (em[1][ph] + ep[1][ph])) * db / (d == 0 ? K.dxi : K.deta);
                }
            }
        } else {
            T w[4][NF];
            for (int q = 0; q < 4; q++)
                for (int k = 0; k < NF; k++) w[q][k] = row[q][k];
            reconstruct(w, uL, uR);
            face_flux_sel(K, P.flags, uL, gW, uR, gC, 0, HXl, kep(i - 1, j, 0), kep(i, j, 0));
            for (int q = 0; q < 4; q++)
                for (int k = 0; k < NF; k++) w[q][k] = row[q + 1][k];
            reconstruct(w, uL, uR);
            face_flux_sel(K, P.flags, uL, gC, uR, gE, 0, HXr, kep(i, j, 0), kep(i + 1, j, 0));
            for (int q = 0; q < 4; q++)
                for (int k = 0; k < NF; k++) w[q][k] = col[q][k];
            reconstruct(w, uL, uR);
            face_flux_sel(K, P.flags, uL, gS, uR, gC, 1, HYb, kep(i, j - 1, 1), kep(i, j, 1));
            for (int q = 0; q < 4; q++)
                for (int k = 0; k < NF; k++) w[q][k] = col[q + 1][k];
            reconstruct(w, uL, uR);
            face_flux_sel(K, P.flags, uL, gC, uR, gN, 1, HYt, kep(i, j, 1), kep(i, j + 1, 1));
        }
        // Mode-II faces, and the flux through every boundary face into its
        // running outflow integral (zero on discharge-inflow faces)
        const double (*inf)[4] = S->inflow[stage_slot(STAGE)];
        constexpr int sl = stage_slot(STAGE);
        // the step's dt (in the state's precision, as the updates use it)
        if (STAGE == 1 && i == 0 && j == 0) bpart[outflow_dt_index(nmax)] = (double)dt;
        if (i == 0) {
            int s = inflow_seg_at(P, 0, j);
            if (s >= 0)
                inflow_flux(K, gC, 0, +1, T(inf[s][0]), T(inf[s][1]), T(inf[s][2]), T(inf[s][3]), HXl);
            put_outflow(bpart, nmax, sl, 0, j, s >= 0 ? 0.0 : -(double)HXl[0] * P.deta,
                        s >= 0 ? 0.0 : -(double)HXl[3] * P.deta);
        }
        if (i == P.nx - 1) {
            int s = inflow_seg_at(P, 1, j);
            if (s >= 0)
                inflow_flux(K, gC, 0, -1, T(inf[s][0]), T(inf[s][1]), T(inf[s][2]), T(inf[s][3]), HXr);
            put_outflow(bpart, nmax, sl, 1, j, s >= 0 ? 0.0 : (double)HXr[0] * P.deta,
                        s >= 0 ? 0.0 : (double)HXr[3] * P.deta);
        }
        if (j == 0) {
            int s = inflow_seg_at(P, 2, i);
            if (s >= 0)
                inflow_flux(K, gC, 1, +1, T(inf[s][0]), T(inf[s][1]), T(inf[s][2]), T(inf[s][3]), HYb);
            put_outflow(bpart, nmax, sl, 2, i, s >= 0 ? 0.0 : -(double)HYb[0] * P.dxi,
                        s >= 0 ? 0.0 : -(double)HYb[3] * P.dxi);
        }
        if (j == P.ny - 1) {
            int s = inflow_seg_at(P, 3, i);
            if (s >= 0)
                inflow_flux(K, gC, 1, -1, T(inf[s][0]), T(inf[s][1]), T(inf[s][2]), T(inf[s][3]), HYt);
            put_outflow(bpart, nmax, sl, 3, i, s >= 0 ? 0.0 : (double)HYt[0] * P.dxi,
                        s >= 0 ? 0.0 : (double)HYt[3] * P.dxi);
        }
        // sources
        const T* uC = row[2];
        T dn[6];
        dn[0] = (gE.nX - gW.nX) / K.two_dxi;
        dn[1] = (gE.nY - gW.nY) / K.two_dxi;
        dn[2] = (gE.nZ - gW.nZ) / K.two_dxi;
        dn[3] = (gN.nX - gS.nX) / K.two_deta;
        dn[4] = (gN.nY - gS.nY) / K.two_deta;
        dn[5] = (gN.nZ - gS.nZ) / K.two_deta;
        T dGx = (fluid_G(row[3][0], row[3][3], gE) - fluid_G(row[1][0], row[1][3], gW)) / K.two_dxi;
        T dGy = (fluid_G(col[3][0], col[3][3], gN) - fluid_G(col[1][0], col[1][3], gS)) / K.two_deta;
        Src<T> Sr;
        sources(K, P.flags, uC, gC, dn, dGx, dGy, Sr, WB ? wbs : nullptr);
        T svx = T(0), svy = T(0);
        if (P.visc) {
            T c9[3][3][NF];
            for (int dj = -1; dj <= 1; dj++)
                for (int di = -1; di <= 1; di++) V.load(i + di, j + dj, c9[dj + 1][di + 1]);
            T u9[3][3], w9[3][3];
            for (int a = 0; a < 3; a++)
                for (int c = 0; c < 3; c++) {
                    dsg2(c9[a][c][4], c9[a][c][5], c9[a][c][3], K.md, u9[a][c], w9[a][c]);
                }
            T JhC = uC[0] + uC[3];
            T JhW = row[1][0] + row[1][3], JhE = row[3][0] + row[3][3];
            T JhS = col[1][0] + col[1][3], JhN = col[3][0] + col[3][3];
            T FX0, FY0, FX1, FY1, GX0, GY0, GX1, GY1;
            // central differences: y-differences at columns i-1, i, i+1 (row j),
            // x-differences at rows j-1, j, j+1 (column i); index [row dj+1][col di+1]
            T cyu[3], cyw[3], cxu[3], cxw[3];
            for (int q = 0; q < 3; q++) {
                cyu[q] = cdiff(u9[2][q], u9[0][q], K.deta);
                cyw[q] = cdiff(w9[2][q], w9[0][q], K.deta);
                cxu[q] = cdiff(u9[q][2], u9[q][0], K.dxi);
                cxw[q] = cdiff(w9[q][2], w9[q][0], K.dxi);
            }
            visc_xface_c(u9[1][0], w9[1][0], u9[1][1], w9[1][1], cyu[0], cyw[0], cyu[1], cyw[1], JhW, JhC, gW, gC,
                         K.dxi, FX0, FY0);
            visc_xface_c(u9[1][1], w9[1][1], u9[1][2], w9[1][2], cyu[1], cyw[1], cyu[2], cyw[2], JhC, JhE, gC, gE,
                         K.dxi, FX1, FY1);
            visc_yface_c(u9[0][1], w9[0][1], u9[1][1], w9[1][1], cxu[0], cxw[0], cxu[1], cxw[1], JhS, JhC, gS, gC,
                         K.deta, GX0, GY0);
            visc_yface_c(u9[1][1], w9[1][1], u9[2][1], w9[2][1], cxu[1], cxw[1], cxu[2], cxw[2], JhC, JhN, gC, gN,
                         K.deta, GX1, GY1);
            T SvX = (FX1 - FX0) / K.dxi + (GX1 - GX0) / K.deta;
            T SvY = (FY1 - FY0) / K.dxi + (GY1 - GY0) / K.deta;
            svx = K.eps * Sr.phif * K.inv_n_r * SvX;
            svy = K.eps * Sr.phif * K.inv_n_r * SvY;
        }
        const size_t c = (size_t)j * P.pitch + i;
        const size_t fs = (size_t)P.ny * P.pitch;
        T tmu = P.has_mu ? mu[c] : K.tan_d;
        T out[NF];
        red[0] = (double)update_cell(K, uC, gC, HXl, HXr, HYb, HYt, Sr, svx, svy, dt, tmu, out,
                                     WB ? cxw : nullptr, WB ? cyw : nullptr);
        if (STAGE > 1) {
#pragma unroll
            for (int k = 0; k < NF; k++) out[k] = stage_combine<STAGE>(Un[k * fs + c], out[k]);
        }
        if (stage_last(STAGE)) {
            T a[2];
            const T km = ep ? ep_kmax(T(P.cos2_int), tmu) : T(1);
            side_speed(K, out, gC, 0, a, km);
            ax = (double)(a[0] > a[1] ? a[0] : a[1]);
            side_speed(K, out, gC, 1, a, km);
            ay = (double)(a[0] > a[1] ? a[0] : a[1]);
        }
#pragma unroll
        for (int k = 0; k < NF; k++) {
            if (stage_last(STAGE) && !isfinite(out[k])) bad = 1;  // as the tiled kernel
            Uout[k * fs + c] = out[k];
        }
    }
    // block reductions (fixed trees: deterministic)
    block_sum<1, 256>(red, sh);
    __syncthreads();
    {
        const int tid = threadIdx.x + threadIdx.y * blockDim.x;
        sh[tid] = ax;
        sh[256 + tid] = ay;
        sh[512 + tid] = bad;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (tid < s) {
                sh[tid] = fmax(sh[tid], sh[tid + s]);
                sh[256 + tid] = fmax(sh[256 + tid], sh[256 + tid + s]);
                sh[512 + tid] = fmax(sh[512 + tid], sh[512 + tid + s]);
            }
            __syncthreads();
        }
        if (tid == 0) {
            const int st = stage_slot(STAGE);
            const int bid = blockIdx.y * gridDim.x + blockIdx.x;
            double* wp = wpart + ((size_t)st * gridDim.x * gridDim.y + bid) * 4;
            wp[0] = sh[0];
            wp[1] = sh[256];
            wp[2] = red[0];
            wp[3] = sh[512];
        }
    }
}

// ---------------------------------------------- earth pressure (option)

// Per cell, the earth-pressure coefficients of the stage input Uin into KE
// ([2][ny][pitch]: K_x, K_y): active in X where the central difference of the
// desingularised solid velocity v_X^s along xi is >= 0, passive otherwise;
// likewise in Y with v_Y^s along eta (neighbours through the ghost map).
template <typename T>
__global__ void __launch_bounds__(256) k_earth_pressure(KParams P, const T* __restrict__ Uin,
                                                        const T* __restrict__ b, const T* __restrict__ mu,
                                                        T* __restrict__ KE)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= P.nx || j >= P.ny) return;
    const Consts<T> K(P);
    const View<T> V(P, Uin, b);
    T uE[NF], uW[NF], uN[NF], uS[NF];
    V.load(i + 1, j, uE);
    V.load(i - 1, j, uW);
    V.load(i, j + 1, uN);
    V.load(i, j - 1, uS);
    const T dvx = dsg(uE[1], uE[0], K.md) - dsg(uW[1], uW[0], K.md);
    const T dvy = dsg(uN[2], uN[0], K.md) - dsg(uS[2], uS[0], K.md);
    const size_t c = (size_t)j * P.pitch + i, fs = (size_t)P.ny * P.pitch;
    const T t = P.has_mu ? mu[c] : K.tan_d;
    const T kx = ep_kx(T(P.cos2_int), t, dvx >= T(0));
    KE[c] = kx;
    KE[fs + c] = ep_ky(kx, t, dvy >= T(0));
}

// ------------------------------------------------------- speeds (init)

template <typename T>
__global__ void __launch_bounds__(256) k_speeds(KParams P, const T* __restrict__ U, const T* __restrict__ b,
                                                const T* __restrict__ mu, double* __restrict__ wpart)
{
    __shared__ double sh[512];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const Consts<T> K(P);
    const View<T> V(P, U, b);
    double ax = 0.0, ay = 0.0;
    if (i < P.nx && j < P.ny) {
        T u[NF], a[2];
        V.load(i, j, u);
        Geo<T> g = V.geo(i, j, K);
        T km = T(1);
        if (P.flags & kFlagEarthPressure)
            km = ep_kmax(T(P.cos2_int), P.has_mu ? mu[(size_t)j * P.pitch + i] : K.tan_d);
        side_speed(K, u, g, 0, a, km);
        ax = (double)(a[0] > a[1] ? a[0] : a[1]);
        side_speed(K, u, g, 1, a, km);
        ay = (double)(a[0] > a[1] ? a[0] : a[1]);
    }
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    sh[tid] = ax;
    sh[256 + tid] = ay;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            sh[tid] = fmax(sh[tid], sh[tid + s]);
            sh[256 + tid] = fmax(sh[256 + tid], sh[256 + tid + s]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        // written into the last stage's slots, which the init finalize reads
        const int bid = blockIdx.y * gridDim.x + blockIdx.x;
        double* wp = wpart + ((size_t)(P.rk - 1) * gridDim.x * gridDim.y + bid) * 4;
        wp[0] = sh[0];
        wp[1] = sh[256];
        wp[2] = 0.0;
        wp[3] = 0.0;
    }
}

// ------------------------------------------------------------- finalize

// Piecewise-linear table lookup: the bracket of tau in the time column
// (held at the end values outside it), then the value of any column.
struct Bracket {
    int k;
    double w;
    bool end;  // tau outside the table: the value is y[k]
};

__device__ __forceinline__ Bracket table_bracket(const double* t, int n, double tau)
{
    if (tau <= t[0]) return {0, 0.0, true};
    if (tau >= t[n - 1]) return {n - 1, 0.0, true};
    int k = 0;
    while (k + 1 < n && t[k + 1] < tau) k++;
    return {k, (tau - t[k]) / (t[k + 1] - t[k]), false};
}

__device__ __forceinline__ double table_at(const double* y, const Bracket& b)
{
    return b.end ? y[b.k] : y[b.k] + b.w * (y[b.k + 1] - y[b.k]);
}


// Cube root of x > 0 to the double whose cube is nearest to x: from the
// device cbrt, step to the neighbour with the smaller exact residual
// |y^3 - x| until neither is smaller (the residual is unimodal, so every
// start ends on the same double; error-free products by fused multiply-add:
// y^2 = p + e, y p = q + f; q - x is exact).  Library cube roots differ by
// units in the last place between platforms; this result does not.
__device__ __forceinline__ double cube_residual(double y, double x)
{
    const double p = y * y;
    const double e = fma(y, y, -p);
    const double q = y * p;
    const double f = fma(y, p, -q);
    const double g = y * e;
    return ((q - x) + f) + g;
}

__device__ __forceinline__ double cbrt_nearest(double x)
{
    double y = cbrt(x);
    if (!(x > 0.0) || !isfinite(x)) return y;
    double r = fabs(cube_residual(y, x));
    for (int it = 0; it < 16; it++) {
        const double lo = nextafter(y, 0.0), hi = nextafter(y, INFINITY);
        const double rl = fabs(cube_residual(lo, x)), rh = fabs(cube_residual(hi, x));
        if (rl < r) {
            y = lo;
            r = rl;
        } else if (rh < r) {
            y = hi;
            r = rh;
        } else {
            break;
        }
    }
    return y;
}

// Critical-depth inflow state of a segment at dimensionless time tau:
// q (discharge per unit width), m_in = (q^2/eps)^(1/3), v_in = q / m_in, phi.
__device__ __forceinline__ void inflow_state(const KParams& P, const double* tables, int s, double tau_nd,
                                             double out[4])
{
    const SegDesc& d = P.seg[s];
    const double* t = tables + d.toff;
    const double* Q = t + d.nt;
    const double* ph = Q + d.nt;
    const Bracket br = table_bracket(t, d.nt, tau_nd * P.T);
    double Qv = table_at(Q, br);
    double phv = table_at(ph, br);
    double w = (d.side < 2) ? P.dy : P.dx;
    double qs = Qv / ((double)d.ncells * w);
    double qn = qs / (P.H * P.V);
    double m = cbrt_nearest(qn * qn / P.eps);
    out[0] = qn;
    out[1] = m;
    out[2] = m > 0.0 ? qn / m : 0.0;
    out[3] = phv;
}

__device__ __forceinline__ double inflow_rate(const KParams& P, const double* tables, double tau, int ph)
{
    double acc = 0.0;
    for (int s = 0; s < P.nseg; s++) {
        double st[4];
        inflow_state(P, tables, s, tau, st);
        double w = (P.seg[s].side < 2) ? P.deta : P.dxi;
        acc += (ph == 0 ? st[3] * st[0] : (1.0 - st[3]) * st[0]) * (double)P.seg[s].ncells * w;
    }
    return acc;
}

// Ghost state of Mode-II state segment s at dimensionless time tau: vertical
// thickness m = h / H and solid fraction phi from the hydrographs, both
// phases moving along the inward normal with speed v; also returns m and v.
__device__ __forceinline__ void ghost_state(const KParams& P, const double* tables, int s, double tau_nd,
                                            double u[NF], double& m_out, double& v_out)
{
    const SegDesc& d = P.sseg[s];
    const double* t = tables + d.toff;
    const double* h = t + d.nt;
    const double* phi = h + d.nt;
    const double* vel = phi + d.nt;
    const Bracket br = table_bracket(t, d.nt, tau_nd * P.T);  // one search for the three columns
    double m = table_at(h, br) / P.H;
    double ph = table_at(phi, br);
    double v = table_at(vel, br) / P.V;
    m_out = m;
    v_out = v;
    double ex = d.side == 0 ? 1.0 : (d.side == 1 ? -1.0 : 0.0);
    double ey = d.side == 2 ? 1.0 : (d.side == 3 ? -1.0 : 0.0);
    double ms = ph * m, mf = (1.0 - ph) * m;
    u[0] = ms;
    u[1] = ms * v * ex;
    u[2] = ms * v * ey;
    u[3] = mf;
    u[4] = mf * v * ex;
    u[5] = mf * v * ey;
}

// values 0, 1 (speed maxima) and 3 (non-finite flag) combine by max, value 2
// (clamp count) by sum
__device__ __forceinline__ bool fin_is_max(int k) { return k != 2; }

// Reduction of the per-wave (or per-block) partial records of a step by one
// workgroup of NT threads into out[kFinVals] (shared memory): the speed
// maxima of the stage that ends the step and the positivity-clamp counts and
// non-finite flags of every stage.  Every thread issues its loads of all
// records together (one memory round trip per batch), then the per-thread
// shares are combined in two short passes over shared memory.  Fixed order
// throughout (deterministic).
template <int NT>
__device__ __forceinline__ void fin_reduce(const KParams& P, int mode, const double* __restrict__ wpart, int nw,
                                           double* out)
{
    constexpr int NCH = NT / 32;  // chunks per value in the first combining pass
    constexpr int CH = NT / NCH;  // shares per chunk
    static_assert(NT % 64 == 0 && NT >= kFinVals * NCH, "finalize workgroup shape");
    __shared__ double sh[kFinVals][NT];
    __shared__ double sh2[kFinVals][NCH];
    const int tid = threadIdx.x;
    const int last = P.rk - 1;  // slot of the stage that ends the step
    {
        double ax = 0.0, ay = 0.0, cl = 0.0, bd = 0.0;
        const double4* wl = reinterpret_cast<const double4*>(wpart) + (size_t)nw * last;  // last stage's slots
        const double4* w0 = reinterpret_cast<const double4*>(wpart);
        const bool two = mode == 0 && last >= 1, three = mode == 0 && last >= 2;
        for (int q0 = tid; q0 < nw; q0 += NT * 8) {
            double4 v[8], e[8], f[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int q = q0 + NT * u;
                const double4 z = make_double4(0.0, 0.0, 0.0, 0.0);
                v[u] = q < nw ? wl[q] : z;
                e[u] = (two && q < nw) ? w0[q] : z;
                f[u] = (three && q < nw) ? w0[(size_t)nw + q] : z;
            }
#pragma unroll
            for (int u = 0; u < 8; u++) {
                ax = fmax(ax, v[u].x);
                ay = fmax(ay, v[u].y);
                cl += v[u].z + e[u].z + f[u].z;
                bd = fmax(bd, fmax(v[u].w, fmax(e[u].w, f[u].w)));
            }
        }
        sh[0][tid] = ax;
        sh[1][tid] = ay;
        sh[2][tid] = cl;
        sh[3][tid] = bd;
    }
    __syncthreads();
    // pass 1: thread (k, c) combines chunk c (CH consecutive shares) of value k
    if (tid < kFinVals * NCH) {
        const int k = tid / NCH, c = tid % NCH;
        const double* r = &sh[k][c * CH];
        double v = r[0];
        if (fin_is_max(k)) {
#pragma unroll 8
            for (int j = 1; j < CH; j++) v = fmax(v, r[j]);
        } else {
#pragma unroll 8
            for (int j = 1; j < CH; j++) v += r[j];
        }
        sh2[k][c] = v;
    }
    __syncthreads();
    // pass 2: thread k combines the chunks of value k
    if (tid < kFinVals) {
        double v = sh2[tid][0];
        for (int c = 1; c < NCH; c++) v = fin_is_max(tid) ? fmax(v, sh2[tid][c]) : v + sh2[tid][c];
        out[tid] = v;
    }
    __syncthreads();
}

// Serial tail of the finalize (one thread), from the reduced values part[]
// (speed maxima, clamp count, non-finite flag).  mode 0: close the step just
// taken (time, inflow integrals; the outflow integrals are kept per boundary
// face by the stage kernels); both modes: next CFL dt from the speed maxima,
// inflow states of the next step's stages, status flags and clamp count.
__device__ __forceinline__ void fin_tail(const KParams& P, DevScalars* S, const double* part,
                                         const double* __restrict__ tables, int mode)
{
    double ax = part[0], ay = part[1];
    if (part[3] > 0.0) S->status |= 1u;
    S->clamps += (unsigned long long)part[2];
    double t = S->t;
    if (mode == 0) {
        const double dt = S->dt;
        const double vs = P.H * P.L * P.L;  // dimensionless volume -> m^3
        for (int ph = 0; ph < 2; ph++) {
            double in;
            if (P.rk == 3) {
                in = dt * (inflow_rate(P, tables, t, ph) / 6.0 + inflow_rate(P, tables, t + dt, ph) / 6.0 +
                           2.0 * inflow_rate(P, tables, t + 0.5 * dt, ph) / 3.0);
            } else {
                in = 0.5 * dt * (inflow_rate(P, tables, t, ph) + inflow_rate(P, tables, t + dt, ph));
            }
            if (ph == 0)
                S->in_s += in * vs;
            else
                S->in_f += in * vs;
        }
        if (dt > 0.0) {
            t += dt;
            S->t = t;
            S->steps += 1;
            S->dt_last = dt;
        }
    }
    for (int s = 0; s < P.nseg; s++) {
        double* st = S->inflow[0][s];  // the first stage's inflow state
        inflow_state(P, tables, s, t, st);
        double a = st[2] + sqrt(P.eps * st[1]);
        if (P.seg[s].side < 2) {
            if (a > ax) ax = a;
        } else if (a > ay)
            ay = a;
    }
    for (int s = 0; s < P.nsseg; s++) {
        double m, v;
        ghost_state(P, tables, s, t, S->sghost[0][s], m, v);  // also the first stage's ghost state
        double a = fabs(v) + sqrt(P.eps * m);
        if (P.sseg[s].side < 2) {
            if (a > ax) ax = a;
        } else if (a > ay)
            ay = a;
    }
    ax = ax > P.a_floor ? ax : P.a_floor;
    ay = ay > P.a_floor ? ay : P.a_floor;
    double dtx = P.dxi / ax, dty = P.deta / ay;
    double dt = P.cfl * (dtx < dty ? dtx : dty);
    if (S->n_sched > 0 && S->steps < S->n_sched) dt = S->dt_sched[S->steps];  // frozen schedule
    if (!isfinite(dt)) S->status |= 1u;
    if (dt < P.dt_floor) S->status |= 2u;
    if (S->t_end - t < dt) dt = S->t_end - t;
    if (dt < 0.0) dt = 0.0;
    S->dt = dt;
    if (S->dt_log) {
        const long long q = S->steps - S->log_base;
        if (q >= 0 && q < S->n_log) S->dt_log[q] = dt;
    }
    // stage times: t, t + dt, and t + dt/2 for the third Runge-Kutta stage
    for (int s = 0; s < P.nseg; s++) {
        inflow_state(P, tables, s, t + dt, S->inflow[1][s]);
        if (P.rk == 3) inflow_state(P, tables, s, t + 0.5 * dt, S->inflow[2][s]);
    }
    for (int s = 0; s < P.nsseg; s++) {
        double m, v;
        ghost_state(P, tables, s, t + dt, S->sghost[1][s], m, v);
        if (P.rk == 3) ghost_state(P, tables, s, t + 0.5 * dt, S->sghost[2][s], m, v);
    }
}

// The tail, run by thread 0 on a copy of the device scalars in shared memory:
// the workgroup loads the record with parallel loads and stores it back the
// same way, so the serial tail does not wait on a memory round trip per field.
__device__ __forceinline__ void fin_tail_staged(const KParams& P, DevScalars* S, const double* red,
                                                const double* __restrict__ tables, int mode)
{
    static_assert(sizeof(DevScalars) % 8 == 0, "device scalars are copied as 8-byte words");
    constexpr int NWORD = sizeof(DevScalars) / 8;
    __shared__ DevScalars Ssh;
    unsigned long long* g = reinterpret_cast<unsigned long long*>(S);
    unsigned long long* l = reinterpret_cast<unsigned long long*>(&Ssh);
    for (int k = threadIdx.x; k < NWORD; k += blockDim.x) l[k] = g[k];
    __syncthreads();
    if (threadIdx.x == 0) fin_tail(P, &Ssh, red, tables, mode);
    __syncthreads();
    for (int k = threadIdx.x; k < NWORD; k += blockDim.x) g[k] = l[k];
}

// Per-step finalize: workgroup 0 reduces the partial records (fixed order),
// then thread 0 runs the tail; in a step (mode 0) the other workgroups, one
// thread per boundary face, add the stages' outflow values to the running
// integrals (launched with 1 + ceil(4 nmax / NT) workgroups).  The hydrograph
// tables of the Mode-II segments are copied into shared memory first when
// they fit (the tail's table lookups are serial searches, each step of which
// would otherwise wait on device memory).
constexpr int kFinTabLds = 2048;

template <typename T, int NT = kFinThreads>
__global__ void __launch_bounds__(NT)
k_finalize(KParams P, DevScalars* S, const double* __restrict__ tables, int mode, const double* __restrict__ wpart,
           int nw, double* __restrict__ bpart, int nmax)
{
    if (blockIdx.x > 0) {
        outflow_accumulate(P, bpart, nmax, (blockIdx.x - 1) * NT + threadIdx.x);
        return;
    }
    __shared__ double red[kFinVals];
    __shared__ double tab[kFinTabLds];
    const bool lds_tab = P.ntab > 0 && P.ntab <= kFinTabLds;
    if (lds_tab)
        for (int k = threadIdx.x; k < P.ntab; k += blockDim.x) tab[k] = tables[k];
    fin_reduce<NT>(P, mode, wpart, nw, red);
    fin_tail_staged(P, S, red, lds_tab ? tab : tables, mode);
}


// ------------------------------------------------- conversions, reductions

// SI fields (device FP64 staging, [7][ny][nx]: h, phi, vxs, vys, vxf, vyf,
// mask of given velocities unused) -> conserved state.
template <typename T>
__global__ void k_set_state(KParams P, const double* __restrict__ f, int vertical, int has_v, T* __restrict__ U,
                            const T* __restrict__ b)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= P.nx || j >= P.ny) return;
    const size_t n = (size_t)P.nx * P.ny, c = (size_t)j * P.nx + i, o = (size_t)j * P.pitch + i;
    const size_t fs = (size_t)P.ny * P.pitch;
    // geometry in FP64 from the FP64 view of the DEM (b may be float)
    auto bv = [&](int ii, int jj) { return (double)b[(size_t)(jj + BHALO) * P.bpitch + BOFF + ii]; };
    Geo<double> g = geometry(bv(i + 1, j), bv(i - 1, j), bv(i, j + 1), bv(i, j - 1), P.two_dxi, P.two_deta);
    double h = f[c], ph = f[n + c];
    double hv = vertical ? h / P.H : g.J * h / P.H;
    double ms = ph * hv, mf = (1.0 - ph) * hv;
    U[0 * fs + o] = T(ms);
    U[1 * fs + o] = T(has_v ? ms * f[2 * n + c] / P.V : 0.0);
    U[2 * fs + o] = T(has_v ? ms * f[3 * n + c] / P.V : 0.0);
    U[3 * fs + o] = T(mf);
    U[4 * fs + o] = T(has_v ? mf * f[4 * n + c] / P.V : 0.0);
    U[5 * fs + o] = T(has_v ? mf * f[5 * n + c] / P.V : 0.0);
}

// conserved state -> SI output fields [6][ny][nx] (h normal, phi_s, velocities)
template <typename T>
__global__ void k_get_fields(KParams P, const T* __restrict__ U, const T* __restrict__ b, double* __restrict__ f)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= P.nx || j >= P.ny) return;
    const size_t n = (size_t)P.nx * P.ny, c = (size_t)j * P.nx + i, o = (size_t)j * P.pitch + i;
    const size_t fs = (size_t)P.ny * P.pitch;
    auto bv = [&](int ii, int jj) { return (double)b[(size_t)(jj + BHALO) * P.bpitch + BOFF + ii]; };
    Geo<double> g = geometry(bv(i + 1, j), bv(i - 1, j), bv(i, j + 1), bv(i, j - 1), P.two_dxi, P.two_deta);
    double ms = (double)U[o], mf = (double)U[3 * fs + o], mt = ms + mf;
    f[c] = mt / g.J * P.H;
    f[n + c] = dsg(ms, mt, P.md);
    f[2 * n + c] = dsg((double)U[1 * fs + o], ms, P.md) * P.V;
    f[3 * n + c] = dsg((double)U[2 * fs + o], ms, P.md) * P.V;
    f[4 * n + c] = dsg((double)U[4 * fs + o], mf, P.md) * P.V;
    f[5 * n + c] = dsg((double)U[5 * fs + o], mf, P.md) * P.V;
}

// FP64 per-block partial volume sums (fixed grid, fixed tree => deterministic).
template <typename T>
__global__ void __launch_bounds__(256) k_mass(KParams P, const T* __restrict__ U, double* __restrict__ part)
{
    __shared__ double sh[2 * 256];
    const size_t n = (size_t)P.nx * P.ny, fs = (size_t)P.ny * P.pitch;
    double a[2] = {0.0, 0.0};
    for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (size_t)gridDim.x * 256) {
        size_t j = c / P.nx, i = c - j * P.nx, o = j * P.pitch + i;
        a[0] += (double)U[o];
        a[1] += (double)U[3 * fs + o];
    }
    sh[threadIdx.x] = a[0];
    sh[256 + threadIdx.x] = a[1];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[threadIdx.x] += sh[threadIdx.x + s];
            sh[256 + threadIdx.x] += sh[256 + threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sh[0];
        part[2 * blockIdx.x + 1] = sh[256];
    }
}

}  // namespace m2p
