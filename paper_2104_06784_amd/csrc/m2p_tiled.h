// m2p_tiled.h -- fused column-marching stage kernel for gfx950.
//
// One wavefront owns a strip of 64 columns (60 output columns plus a halo of
// two on each side) and marches up R rows.  The y-direction stencil of the
// scheme (minmod slopes need rows j-1..j+2, sources and viscosity rows
// j-1..j+1) lives in a rolling register window; x-neighbours are exchanged by
// cross-lane shuffles.  Every face flux, every cell geometry and every
// derived cell quantity is computed once per stage (the y-face flux of row
// j+1/2 is carried to the next row), so the kernel reads each state field
// once per row from HBM and the march needs no LDS and no barrier (one
// barrier at the end combines a workgroup's partial sums).  The arithmetic of
// every quantity is the one of m2p_device.h in the same order as the
// reference kernel, so FP64 results are bitwise identical to it (the FP32
// stage 1 carries face fluxes as 2 H, see carry_2h).  In FP32 the quantities
// a row block's prologue recomputes (row geometry, slopes, the face flux
// below the block) are fused the same way as in the march, so FP32 results
// do not depend on the tile height either.
#pragma once

#include "m2p_device.h"
#include "m2p_launch.h"

namespace m2p {

constexpr int kStripOut = 60;  // output columns per wavefront

// Wavefront-wide shifts by one lane with DPP (wave_shl:1 / wave_shr:1, a
// VALU move with no LDS round trip).  The edge lane without a source gets 0
// from the bound control (no zeroed destination register needed first);
// edge lanes are halo lanes whose results never reach an output column.
__device__ __forceinline__ int dpp_right_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ int dpp_left_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }

__device__ __forceinline__ float from_right(float v) { return __int_as_float(dpp_right_i(__float_as_int(v))); }
__device__ __forceinline__ float from_left(float v) { return __int_as_float(dpp_left_i(__float_as_int(v))); }

__device__ __forceinline__ double from_right(double v)
{
    const long long x = __double_as_longlong(v);
    const int lo = dpp_right_i((int)(x & 0xffffffffll)), hi = dpp_right_i((int)(x >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double from_left(double v)
{
    const long long x = __double_as_longlong(v);
    const int lo = dpp_left_i((int)(x & 0xffffffffll)), hi = dpp_left_i((int)(x >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Raw buffer access: the array's base in a scalar resource, a field's offset
// in a scalar register and the cell's byte offset in one 32-bit lane
// register, so a load or store needs no 64-bit address arithmetic (which a
// global access spends one VALU instruction on).  Offsets must stay below
// 2 GiB.  Word 3 is the gfx9-family raw-buffer format.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t brsrc(const void* p)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ float bload(float*, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
}
__device__ __forceinline__ double bload(double*, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0));
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)vo, (int)so, 0);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so)
{
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)vo, (int)so, 0);
}

// Per-row quantities kept in the rolling window.
template <typename T>
struct RowD {
    Geo<T> g;      // basal geometry of the cell
    T u, w;        // fluid velocities (desingularised)
    T cdxu, cdxw;  // central x-differences of u, w
    T Jh;          // J_b h = m^s + m^f
    T Gf;          // J_b h pbar^f
    T kx, ky;      // earth-pressure coefficients of the stage input (the option; else unused)
    T cx;          // well-balanced option: c with the bed of both x-neighbours from memory (else unused)
};

// Earth-pressure coefficients for a uniform basal friction t: K_x active and
// passive, K_y for each K_x and each sign of the y-difference (kyap: K_x
// active, K_y passive), computed once by the per-cell functions; kypp is also
// the CFL bound ep_kmax.
template <typename T>
struct EPTab {
    T kxa, kxp, kyaa, kyap, kypa, kypp;
    __device__ __forceinline__ void init(T c2, T t)
    {
        kxa = ep_kx(c2, t, true);
        kxp = ep_kx(c2, t, false);
        kyaa = ep_ky(kxa, t, true);
        kyap = ep_ky(kxa, t, false);
        kypa = ep_ky(kxp, t, true);
        kypp = ep_ky(kxp, t, false);
    }
};

// Well-balanced option: a row's face values along y (eta per phase and the
// bed, minus and plus side) and the right-cell pressure correction of the
// y-face below it (momentum components 1, 2, 4, 5), carried up the march.
template <typename T>
struct WBRow {
    T em[2], ep[2], bm, bp, sb;  // sb: the bed slope along y
    T cr[4];
};

// Face values along one direction of a cell from the masses m0..m2 of phase
// ph's three cells along it, their c^2 and beds (wb_cell on eta = eps c^2 m).
template <typename T>
__device__ __forceinline__ void wb_row_values(const Consts<T>& K, const T* u0, const T* u1, const T* u2, T c0, T c1,
                                              T c2, T b0, T b1, T b2, WBRow<T>& w)
{
#pragma unroll
    for (int ph = 0; ph < 2; ph++) {
        T bm, bp, sb;
        wb_cell(K.eps * (c0 * c0) * u0[3 * ph], K.eps * (c1 * c1) * u1[3 * ph], K.eps * (c2 * c2) * u2[3 * ph], b0, b1,
                b2, w.em[ph], w.ep[ph], bm, bp, &sb);
        w.bm = bm;
        w.bp = bp;
        w.sb = sb;
    }
}

// With EP, also the row's earth-pressure coefficients from the solid
// velocities of its x-neighbours (lane shifts) and of the rows below (uS) and
// above (uN), with the cell's basal friction tmu -- the arithmetic of the
// coefficient pass k_earth_pressure (with a uniform friction, uni, the
// coefficients come from tab).
template <typename T, bool EP = false>
__device__ __forceinline__ void make_row(const Consts<T>& K, const T u[NF], T bC, T bS, T bN, RowD<T>& r,
                                         const T* uS = nullptr, const T* uN = nullptr, T c2 = T(0), T tmu = T(0),
                                         bool uni = false, const EPTab<T>* tab = nullptr)
{
    const T bE = from_right(bC), bW = from_left(bC);
    r.g = geometry(bE, bW, bN, bS, K.two_dxi, K.two_deta);
    dsg2(u[4], u[5], u[3], K.md, r.u, r.w);
    const T uE = from_right(r.u), uW = from_left(r.u);
    const T wE = from_right(r.w), wW = from_left(r.w);
    r.cdxu = cdiff(uE, uW, K.dxi);
    r.cdxw = cdiff(wE, wW, K.dxi);
    r.Jh = u[0] + u[3];
    r.Gf = fluid_G(u[0], u[3], r.g);
    if constexpr (EP) {
        const T vxs = dsg(u[1], u[0], K.md);
        const T dvx = from_right(vxs) - from_left(vxs);
        const T dvy = dsg(uN[2], uN[0], K.md) - dsg(uS[2], uS[0], K.md);
        if (uni) {
            r.kx = dvx >= T(0) ? tab->kxa : tab->kxp;
            r.ky = dvx >= T(0) ? (dvy >= T(0) ? tab->kyaa : tab->kyap) : (dvy >= T(0) ? tab->kypa : tab->kypp);
        } else {
            r.kx = ep_kx(c2, tmu, dvx >= T(0));
            r.ky = ep_ky(r.kx, tmu, dvy >= T(0));
        }
    }
}

template <typename T>
__device__ __forceinline__ void visc_yface_rows(const RowD<T>& a, const RowD<T>& b, const Consts<T>& K, T& GX, T& GY)
{
    visc_yface_c(a.u, a.w, b.u, b.w, a.cdxu, a.cdxw, b.cdxu, b.cdxw, a.Jh, b.Jh, a.g, b.g, K.deta, GX, GY);
}

// Occupancy hint of the FP32 single-scenario stage kernels (waves per SIMD
// the register allocation must allow; 1 = no constraint).  Three waves (at
// most 168 VGPRs) for every FP32 stage: they fit without spilling and the
// later stages (which also carry U^n and the CFL speeds) run 8 % faster than
// at two waves.  The FP64 kernels and the batched kernels keep the
// compiler's choice.
#ifndef M2P_TILED_WPE_S1
#define M2P_TILED_WPE_S1 3
#endif
#ifndef M2P_TILED_WPE_S2
#define M2P_TILED_WPE_S2 3
#endif
// The earth-pressure instance carries the coefficients of three rows
// besides; it fits three waves (its last stages with 6 VGPRs spilled, 9 %
// faster per step than at two waves) because its march reads the cell's own
// U^n just before the update and prefetches row j + 3 after the row's stores
// (both held across the whole row otherwise).
#ifndef M2P_TILED_WPE_EP
#define M2P_TILED_WPE_EP 3
#endif
// The well-balanced instance carries the face values and corrections of the
// hydrostatic reconstruction besides: two waves.
#ifndef M2P_TILED_WPE_WB
#define M2P_TILED_WPE_WB 2
#endif
template <typename T, int STAGE, bool EP = false, bool WB = false>
constexpr int tiled_wpe()
{
    return sizeof(T) == 4
               ? (WB ? M2P_TILED_WPE_WB
                     : (EP ? M2P_TILED_WPE_EP : (STAGE == 1 ? M2P_TILED_WPE_S1 : M2P_TILED_WPE_S2)))
               : 1;
}

// Partials of one wavefront's share of a stage: speed maxima (last stage),
// positivity-clamp count, non-finite flag.
struct WavePart {
    double ax, ay, cl, bd;
};

// One wavefront's share of a stage: strip `strip`, row block `rb` of one
// scenario; returns its partials (the same in every lane).  GH: the
// scenario has Mode-II state segments, whose ghost cells replace the mapped
// boundary values (a separate instance, so runs without them carry none of
// that code in the march).  CU: central-upwind face fluxes.  EP: Savage-Hutter
// earth-pressure coefficients, computed in the march for the row ahead (a
// ghost cell takes those of the cell it maps to).  BUF: the state and DEM
// accesses as raw buffer accesses (every byte offset below 2 GiB; 3 % faster
// per step at 4096 x 4096).  WB: the well-balanced hydrostatic reconstruction
// (Mode-I, no earth pressure; the face flux the flags select).
template <typename T, int STAGE, bool GH, bool CU = false, bool EP = false, bool BUF = false, bool WB = false>
__device__ __forceinline__ WavePart stage_tiled_wave(const KParams& P, const T* __restrict__ Uin, const T* Un, T* Uout,
                                                 const T* __restrict__ b, const T* __restrict__ mu,
                                                 DevScalars* __restrict__ S, double* __restrict__ bpart,
                                                 int nmax, int R, int nstrips, int nrb, int strip, int rb, int lane)
{
    const Consts<T> K(P);
    // stage 1 carries face fluxes as 2 H in the FP32 forms (later stages keep
    // H: the extra registers of the factorised update do not fit their
    // three-waves-per-SIMD budget)
    constexpr bool H2 = STAGE == 1 && !WB;
    const size_t fs = (size_t)P.ny * P.pitch;
    const int col = strip * kStripOut - 2 + lane;
    const int cc = col < P.nx + 1 ? col : P.nx + 1;  // lanes past the ghost ring feed no output
    int fx = 0;
    const int mi = map_index(cc, P.nx, P.bc[0], P.bc[1], fx);
    const int bcol = BOFF + cc;
    const bool out_lane = lane >= 2 && lane < 62 && col < P.nx;
    const int r0 = rb * R;
    const int r1 = r0 + R < P.ny ? r0 + R : P.ny;
    const T dt = T(S->dt);
    const double(*inf)[4] = S->inflow[stage_slot(STAGE)];
    const bool ownW = out_lane && col == 0;  // this lane owns the W / E boundary face
    const bool ownE = out_lane && col == P.nx - 1;
    // side whose ghost columns this strip holds when it holds one side's only
    // (wave-uniform): W for the first strip, E for the last, else none
    const int edge_side = nstrips == 1 ? -1 : (strip == 0 ? 0 : (strip == nstrips - 1 ? 1 : -1));

    const __amdgpu_buffer_rsrc_t rU = brsrc(Uin), rN = brsrc(Un), rO = brsrc(Uout), rB = brsrc(b);
    const unsigned fsb = (unsigned)(fs * sizeof(T));
    auto loadU = [&](int r, T u[NF]) {
        int fy = 0;
        const int mj = map_index(r, P.ny, P.bc[2], P.bc[3], fy);
        const size_t o = (size_t)mj * P.pitch + mi;
#pragma unroll
        for (int k = 0; k < NF; k++) {
            if constexpr (BUF)
                u[k] = bload((T*)nullptr, rU, (unsigned)(o * sizeof(T)), k * fsb);
            else
                u[k] = Uin[k * fs + o];
        }
        if (fx) {
            u[1] = -u[1];
            u[4] = -u[4];
        }
        if (fy) {
            u[2] = -u[2];
            u[5] = -u[5];
        }
        // only cells outside the grid can be ghosts of a state segment (for
        // interior strips and rows the branch is skipped by the whole wave).
        // The W / E ghost columns of an edge strip in a grid row all face one
        // segment, found from wave-uniform values, so its state is read with
        // scalar loads; ghost rows and single-strip grids take the general
        // per-lane lookup.
        if constexpr (GH) {
            const bool grow = (unsigned)r >= (unsigned)P.ny;
            const bool gcol = (unsigned)cc >= (unsigned)P.nx;
            if (!grow && edge_side >= 0) {
                if (gcol) {
                    const int sg = state_seg_at(P, edge_side, r);
                    if (sg >= 0) {
                        const double* g = S->sghost[stage_slot(STAGE)][sg];
#pragma unroll
                        for (int k = 0; k < NF; k++) u[k] = T(g[k]);
                    }
                }
            } else if (grow || gcol) {
                ghost_sub(P, S->sghost[stage_slot(STAGE)], cc, r, u);
            }
        }
    };
    auto loadB = [&](int r) {
        const size_t o = (size_t)(r + BHALO) * P.bpitch + bcol;
        if constexpr (BUF)
            return bload((T*)nullptr, rB, (unsigned)(o * sizeof(T)), 0u);
        else
            return b[o];
    };
    // Well-balanced option: the eta slopes along x of lanes 1 and 62 need c
    // of lanes 0 and 63, whose geometry took one x-neighbour's bed from
    // outside the wavefront; those two lanes recompute c with that bed read
    // from memory (a column of the padded DEM row, clamped into the row).
    auto wb_cx = [&](int r, T bC, T bS, T bN, RowD<T>& D) {
        if constexpr (WB) {
            const T bE = from_right(bC), bW = from_left(bC);
            D.cx = D.g.c;
            if (lane == 0 || lane == 63) {
                const int c = bcol + (lane == 0 ? -1 : 1);
                const size_t o = (size_t)(r + BHALO) * P.bpitch + (c < P.bpitch ? c : P.bpitch - 1);
                T bo;
                if constexpr (BUF)
                    bo = bload((T*)nullptr, rB, (unsigned)(o * sizeof(T)), 0u);
                else
                    bo = b[o];
                D.cx = geometry(lane == 63 ? bo : bE, lane == 0 ? bo : bW, bN, bS, K.two_dxi, K.two_deta).c;
            }
        }
    };

    // flux through each boundary face into the stage's outflow slot (zero on
    // discharge-inflow faces); the first stage records the step the updates
    // use (dt in the state's precision: the volume that left the cells)
    if (STAGE == 1 && strip == 0 && rb == 0 && lane == 0) bpart[outflow_dt_index(nmax)] = (double)dt;
    auto put_b = [&](int side, int k, bool inflow, T m_s, T m_f, double len) {
        constexpr double unit = carry_2h<T, H2>() ? 0.5 : 1.0;
        const double sg = (side == 0 || side == 2) ? -unit : unit;
        put_outflow(bpart, nmax, stage_slot(STAGE), side, k,
                    inflow ? 0.0 : sg * (double)m_s * len, inflow ? 0.0 : sg * (double)m_f * len);
    };
    T amx = T(0), amy = T(0);
    int clamps = 0, bad = 0;

    // ---- prologue: rows r0-2 .. r0+1
    T Um2[NF], Um1[NF], U0[NF], U1[NF];
    loadU(r0 - 2, Um2);
    loadU(r0 - 1, Um1);
    loadU(r0, U0);
    loadU(r0 + 1, U1);
    T bm2 = loadB(r0 - 2), bm1 = loadB(r0 - 1), b0 = loadB(r0), b1 = loadB(r0 + 1);
    RowD<T> Dm, D0;  // rows j-1, j
    const T c2 = T(P.cos2_int);
    // basal friction of row r (the earth-pressure coefficients need it)
    auto tmu_row = [&](int r) {
        if (!P.has_mu) return K.tan_d;
        int f = 0;
        return mu[(size_t)map_index(r, P.ny, P.bc[2], P.bc[3], f) * P.pitch + mi];
    };
    // lanes of the ghost columns next to the edges take the coefficient of
    // the edge cell they map to (the lanes further out feed no used face)
    const bool ghostW = col == -1, ghostE = col == P.nx;
    const bool uni = !P.has_mu;
    EPTab<T> tab;
    if (EP && uni) tab.init(c2, K.tan_d);
    make_row<T, EP>(K, Um1, bm1, bm2, b0, Dm, Um2, U0, c2, EP && !uni ? tmu_row(r0 - 1) : T(0), uni, &tab);
    make_row<T, EP>(K, U0, b0, bm1, b1, D0, Um1, U1, c2, EP && !uni ? tmu_row(r0) : T(0), uni, &tab);
    wb_cx(r0 - 1, bm1, bm2, b0, Dm);
    wb_cx(r0, b0, bm1, b1, D0);
    if (EP && r0 == 0) Dm.ky = D0.ky;  // ghost row -1 maps to row 0
    T sy0[NF];  // y-slopes of row r0
    T Hy[NF];            // y-face flux j - 1/2
    WBRow<T> wa, wb;     // well-balanced carries, slot (row - r0) mod 2
    {
        T sym[NF], uL[NF], uR[NF];
#pragma unroll
        for (int k = 0; k < NF; k++) {
            sym[k] = minmod(Um1[k] - Um2[k], U0[k] - Um1[k]);
            sy0[k] = minmod(U0[k] - Um1[k], U1[k] - U0[k]);
            uL[k] = Um1[k] + T(0.5) * sym[k];
            uR[k] = U0[k] - T(0.5) * sy0[k];
        }
        if constexpr (WB) {
            // face values of rows r0 - 1 and r0: c of row r0 - 2 (the ghost row
            // -2 takes row -1's) and of row r0 + 1 from their geometry
            const T bm3 = r0 - 2 < -1 ? T(0) : loadB(r0 - 3);
            const T cm2 = r0 - 2 < -1 ? Dm.g.c
                                      : geometry(from_right(bm2), from_left(bm2), bm1, bm3, K.two_dxi, K.two_deta).c;
            const T b2 = loadB(r0 + 2);
            const T c1 = geometry(from_right(b1), from_left(b1), b2, b0, K.two_dxi, K.two_deta).c;
            WBRow<T> wm;
            wb_row_values(K, Um2, Um1, U0, cm2, Dm.g.c, D0.g.c, bm2, bm1, b0, wm);
            wb_row_values(K, Um1, U0, U1, Dm.g.c, D0.g.c, c1, bm1, b0, b1, wa);
            const T wmb[2] = {wm.bp, wm.bp}, wab[2] = {wa.bm, wa.bm};
            T cl[NF], cr[NF];
            wb_face(K, P.flags, uL, Dm.g, Dm.g.c * Dm.g.c, uR, D0.g, D0.g.c * D0.g.c, wm.ep, wmb, wa.em, wab,
                    wb_bed_jump(bm1, b0, wm.sb, wa.sb), r0 == 0 && P.bc[2] == 1, false, 1, Hy, cl, cr);
            wa.cr[0] = cr[1];
            wa.cr[1] = cr[2];
            wa.cr[2] = cr[4];
            wa.cr[3] = cr[5];
        } else {
            central_flux<T, H2, CU>(K, uL, Dm.g, uR, D0.g, 1, Hy, EP ? Dm.ky : T(1), EP ? D0.ky : T(1));
        }
        if (r0 == 0 && out_lane) {
            const int s = inflow_seg_at(P, 2, col);
            if (s >= 0)
                inflow_flux<T, H2>(K, D0.g, 1, +1, T(inf[s][0]), T(inf[s][1]), T(inf[s][2]), T(inf[s][3]), Hy);
            put_b(2, col, s >= 0, Hy[0], Hy[3], P.dxi);
        }
    }
    // viscous y-face j - 1/2
    T vGX = T(0), vGY = T(0);
    if (P.visc)
        visc_yface_rows(Dm, D0, K, vGX, vGY);
    T Ua[NF], Ub[NF], Uc_[NF], Ud[NF];  // U rows, slot (row - r0) mod 4
    RowD<T> Da, Db, Dc, Dd;            // row quantities, same slot rule
    T sya[NF], syb[NF], Hya[NF], Hyb[NF];
    T vGXa = vGX, vGYa = vGY, vGXb = T(0), vGYb = T(0);
#pragma unroll
    for (int k = 0; k < NF; k++) {
        Ua[k] = U0[k];
        Ub[k] = U1[k];
        sya[k] = sy0[k];
        Hya[k] = Hy[k];
    }
    Da = D0;
    Dd = Dm;
    loadU(r0 + 2, Uc_);
    T ba = b0, bb = b1, bc = loadB(r0 + 2), bd = T(0);

    // One row j.  Uc, Un1, U2: rows j..j+2; U3, bj3 receive row j+3.  Dm, D0:
    // rows j-1, j; D1 receives row j+1.  sy0, Hy, vGX/vGY: y-slopes of row j,
    // flux and viscous flux of face j-1/2; sy1, HyN, vGXN/vGYN receive those
    // of row j+1 / face j+1/2.  The march calls it with the slots rotated, so
    // the window never moves through registers.
    auto row = [&](int j, T* Uc, T* Un1, T* U2, T* U3, T bj, T bj1, T bj2, T& bj3, RowD<T>& Dm, RowD<T>& D0,
                   RowD<T>& D1, T* sy0, T* sy1, T* Hy, T* HyN, T vGX, T vGY, T& vGXN, T& vGYN, WBRow<T>& w0,
                   WBRow<T>& w1) __attribute__((always_inline)) {
        // ---- prefetch row j+3 (consumed next iteration) and this row's own
        // values needed at the end (U^n for the Heun average, tan delta);
        // the earth-pressure instance reads them where they are used instead
        // (fewer registers held across the row: it then fits three waves)
        const int rn = j + 3 <= P.ny + 1 ? j + 3 : P.ny + 1;
        if (!EP) {
            loadU(rn, U3);
            bj3 = loadB(rn);
        }
        const size_t cself = (size_t)j * P.pitch + (out_lane ? col : 0);
        T unr[NF];
        auto load_un = [&]() {
#pragma unroll
            for (int k = 0; k < NF; k++) {
                if constexpr (BUF)
                    unr[k] = bload((T*)nullptr, rN, (unsigned)(cself * sizeof(T)), k * fsb);
                else
                    unr[k] = Un[k * fs + cself];
            }
        };
        if (STAGE > 1 && !EP) load_un();
        const T tmu = P.has_mu ? mu[cself] : K.tan_d;
        make_row<T, EP>(K, Un1, bj1, bj, bj2, D1, Uc, U2, c2, EP && !uni ? tmu_row(j + 1) : T(0), uni, &tab);
        wb_cx(j + 1, bj1, bj, bj2, D1);
        if (EP && j + 1 == P.ny) D1.ky = D0.ky;  // ghost row ny maps to row ny - 1
        T uL[NF], uR[NF];
#pragma unroll
        for (int k = 0; k < NF; k++) {
            sy1[k] = minmod(Un1[k] - Uc[k], U2[k] - Un1[k]);
            uL[k] = Uc[k] + T(0.5) * sy0[k];
            uR[k] = Un1[k] - T(0.5) * sy1[k];
        }
        // ---- y-face j + 1/2
        T cy[NF];  // well-balanced: the cell's y corrections
        if constexpr (WB) {
            // face values of row j + 1 (c of row j + 2 from its geometry; the
            // ghost row ny + 1 takes row ny's)
            const T cj2 = j + 2 > P.ny ? D1.g.c
                                       : geometry(from_right(bj2), from_left(bj2), bj3, bj1, K.two_dxi, K.two_deta).c;
            wb_row_values(K, Uc, Un1, U2, D0.g.c, D1.g.c, cj2, bj, bj1, bj2, w1);
            const T w0b[2] = {w0.bp, w0.bp}, w1b[2] = {w1.bm, w1.bm};
            T cl[NF], cr[NF];
            wb_face(K, P.flags, uL, D0.g, D0.g.c * D0.g.c, uR, D1.g, D1.g.c * D1.g.c, w0.ep, w0b, w1.em, w1b,
                    wb_bed_jump(bj, bj1, w0.sb, w1.sb), false, j + 1 == P.ny && P.bc[3] == 1, 1, HyN, cl, cr);
            cy[0] = T(0);
            cy[1] = cl[1] - w0.cr[0];
            cy[2] = cl[2] - w0.cr[1];
            cy[3] = T(0);
            cy[4] = cl[4] - w0.cr[2];
            cy[5] = cl[5] - w0.cr[3];
            w1.cr[0] = cr[1];
            w1.cr[1] = cr[2];
            w1.cr[2] = cr[4];
            w1.cr[3] = cr[5];
        } else {
            central_flux<T, H2, CU>(K, uL, D0.g, uR, D1.g, 1, HyN, EP ? D0.ky : T(1), EP ? D1.ky : T(1));
        }
        if (j == P.ny - 1 && out_lane) {
            const int s = inflow_seg_at(P, 3, col);
            if (s >= 0)
                inflow_flux<T, H2>(K, D0.g, 1, -1, T(inf[s][0]), T(inf[s][1]), T(inf[s][2]), T(inf[s][3]), HyN);
            put_b(3, col, s >= 0, HyN[0], HyN[3], P.dxi);
        }
        vGXN = T(0);
        vGYN = T(0);
        if (P.visc) visc_yface_rows(D0, D1, K, vGXN, vGYN);

        // ---- x-faces of row j: this lane computes face i + 1/2
        T Hx[NF], HxL[NF];
        T cxw[NF], wbs[4];  // well-balanced: the cell's x corrections, balanced source terms
        {
            T sx[NF], up[NF], um[NF], upR[NF];
#pragma unroll
            for (int k = 0; k < NF; k++) {
                const T wE = from_right(Uc[k]), wW = from_left(Uc[k]);
                sx[k] = minmod(Uc[k] - wW, wE - Uc[k]);
                um[k] = Uc[k] + T(0.5) * sx[k];  // left value of face i + 1/2
                up[k] = Uc[k] - T(0.5) * sx[k];  // right value of face i - 1/2
            }
#pragma unroll
            for (int k = 0; k < NF; k++) upR[k] = from_right(up[k]);
            Geo<T> gR;
            gR.bX = from_right(D0.g.bX);
            gR.bY = from_right(D0.g.bY);
            gR.J = from_right(D0.g.J);
            gR.c = from_right(D0.g.c);
            gR.nX = gR.nY = gR.nZ = T(0);
            gR.A11 = from_right(D0.g.A11);
            gR.A12 = from_right(D0.g.A12);
            gR.A21 = gR.A12;
            gR.A22 = from_right(D0.g.A22);
            T kL = T(1), kR = T(1);
            if constexpr (EP) {
                const T fromE = from_right(D0.kx), fromW = from_left(D0.kx);
                kL = ghostW ? fromE : (ghostE ? fromW : D0.kx);
                kR = from_right(kL);
            }
            if constexpr (WB) {
                // c along x: a column two outside takes the ghost column's
                const T cE = from_right(D0.cx), cW = from_left(D0.cx);
                const T cx = col <= -2 ? cE : (col >= P.nx + 1 ? cW : D0.cx);
                const T c2x = cx * cx;
                const T bE = from_right(bj), bW = from_left(bj);
                T em[2], ep[2], bm[2], bp[2], emR[2], bmR[2], sb = T(0);
#pragma unroll
                for (int ph = 0; ph < 2; ph++) {
                    const T e = K.eps * c2x * Uc[3 * ph];
                    wb_cell(from_left(e), e, from_right(e), bW, bj, bE, em[ph], ep[ph], bm[ph], bp[ph], &sb);
                    emR[ph] = from_right(em[ph]);
                    bmR[ph] = from_right(bm[ph]);
                }
                T cl[NF], cr[NF];
                wb_face(K, P.flags, um, D0.g, c2x, upR, gR, from_right(c2x), ep, bp, emR, bmR,
                        wb_bed_jump(bj, bE, sb, from_right(sb)), col == -1 && P.bc[0] == 1,
                        col + 1 == P.nx && P.bc[1] == 1, 0, Hx, cl, cr);
                cxw[0] = T(0);
                cxw[3] = T(0);
#pragma unroll
                for (int k = 1; k < NF; k++)
                    if (k != 3) cxw[k] = cl[k] - from_left(cr[k]);
#pragma unroll
                for (int ph = 0; ph < 2; ph++) {
                    const T fac = ph == 0 ? T(1) - K.al : T(1);
                    // (the FP32 forms take the bed slopes themselves for the face differences)
                    const T dbx = Folded<T>::value ? sb : bp[ph] - bm[ph];
                    const T dby = Folded<T>::value ? w0.sb : w0.bp - w0.bm;
                    wbs[2 * ph] = -(fac / K.eps) * (T(0.5) * (em[ph] + ep[ph])) * dbx / K.dxi;
                    wbs[2 * ph + 1] = -(fac / K.eps) * (T(0.5) * (w0.em[ph] + w0.ep[ph])) * dby / K.deta;
                }
            } else {
                central_flux<T, H2, CU>(K, um, D0.g, upR, gR, 0, Hx, kL, kR);
            }
#pragma unroll
            for (int k = 0; k < NF; k++) HxL[k] = from_left(Hx[k]);
        }
        if (ownW) {
            const int s = inflow_seg_at(P, 0, j);
            if (s >= 0)
                inflow_flux<T, H2>(K, D0.g, 0, +1, T(inf[s][0]), T(inf[s][1]), T(inf[s][2]), T(inf[s][3]), HxL);
            put_b(0, j, s >= 0, HxL[0], HxL[3], P.deta);
        }
        if (ownE) {
            const int s = inflow_seg_at(P, 1, j);
            if (s >= 0)
                inflow_flux<T, H2>(K, D0.g, 0, -1, T(inf[s][0]), T(inf[s][1]), T(inf[s][2]), T(inf[s][3]), Hx);
            put_b(1, j, s >= 0, Hx[0], Hx[3], P.deta);
        }

        // ---- sources of row j
        T dn[6];
        {
            const T nXE = from_right(D0.g.nX), nXW = from_left(D0.g.nX);
            const T nYE = from_right(D0.g.nY), nYW = from_left(D0.g.nY);
            const T nZE = from_right(D0.g.nZ), nZW = from_left(D0.g.nZ);
            dn[0] = (nXE - nXW) / K.two_dxi;
            dn[1] = (nYE - nYW) / K.two_dxi;
            dn[2] = (nZE - nZW) / K.two_dxi;
            dn[3] = (D1.g.nX - Dm.g.nX) / K.two_deta;
            dn[4] = (D1.g.nY - Dm.g.nY) / K.two_deta;
            dn[5] = (D1.g.nZ - Dm.g.nZ) / K.two_deta;
        }
        const T GE = from_right(D0.Gf), GW = from_left(D0.Gf);
        const T dGx = (GE - GW) / K.two_dxi;
        const T dGy = (D1.Gf - Dm.Gf) / K.two_deta;
        Src<T> Sr;
        sources(K, P.flags, Uc, D0.g, dn, dGx, dGy, Sr, WB ? wbs : nullptr);
        T svx = T(0), svy = T(0);
        if (P.visc) {
            // x-face i + 1/2 viscous fluxes, then face i - 1/2 from the left lane
            const T cdyu = cdiff(D1.u, Dm.u, K.deta);
            const T cdyw = cdiff(D1.w, Dm.w, K.deta);
            const T uE = from_right(D0.u), wE = from_right(D0.w);
            const T cdyuE = from_right(cdyu), cdywE = from_right(cdyw);
            const T JhE = from_right(D0.Jh);
            Geo<T> gE;
            gE.A11 = from_right(D0.g.A11);
            gE.A12 = from_right(D0.g.A12);
            gE.A21 = gE.A12;
            gE.A22 = from_right(D0.g.A22);
            T FX1, FY1;
            visc_xface_c(D0.u, D0.w, uE, wE, cdyu, cdyw, cdyuE, cdywE, D0.Jh, JhE, D0.g, gE, K.dxi, FX1, FY1);
            const T FX0 = from_left(FX1), FY0 = from_left(FY1);
            const T SvX = (FX1 - FX0) / K.dxi + (vGXN - vGX) / K.deta;
            const T SvY = (FY1 - FY0) / K.dxi + (vGYN - vGY) / K.deta;
            svx = K.eps * Sr.phif * K.inv_n_r * SvX;
            svy = K.eps * Sr.phif * K.inv_n_r * SvY;
        }
        // ---- update and write
        if (out_lane) {
            T out[NF];
            clamps += update_cell<T, H2, false>(K, Uc, D0.g, HxL, Hx, Hy, HyN, Sr, svx, svy, dt, tmu, out,
                                                WB ? cxw : nullptr, WB ? cy : nullptr);
            if (STAGE > 1) {
                if (EP) load_un();
#pragma unroll
                for (int k = 0; k < NF; k++) out[k] = stage_combine<STAGE>(unr[k], out[k]);
            }
            if (stage_last(STAGE)) {
                T sx, sy;
                cell_speeds(K, out, D0.g, sx, sy, EP ? (uni ? tab.kypp : ep_kmax(c2, tmu)) : T(1));
                amx = fmax(amx, sx);
                amy = fmax(amy, sy);
            }
            // non-finite check in the stage that ends the step only: a value
            // that is not finite after an earlier stage reaches its output
#pragma unroll
            for (int k = 0; k < NF; k++) {
                if (stage_last(STAGE) && !isfinite(out[k])) bad = 1;
                if constexpr (BUF)
                    bstore(out[k], rO, (unsigned)(cself * sizeof(T)), k * fsb);
                else
                    Uout[k * fs + cself] = out[k];
            }
        }
        if (EP) {
            loadU(rn, U3);
            bj3 = loadB(rn);
        }
    };

    // rows r0 .. r1-1, four per trip with the slots rotated
    for (int j = r0; j < r1; j += 4) {
        row(j, Ua, Ub, Uc_, Ud, ba, bb, bc, bd, Dd, Da, Db, sya, syb, Hya, Hyb, vGXa, vGYa, vGXb, vGYb, wa, wb);
        if (j + 1 >= r1) break;
        row(j + 1, Ub, Uc_, Ud, Ua, bb, bc, bd, ba, Da, Db, Dc, syb, sya, Hyb, Hya, vGXb, vGYb, vGXa, vGYa, wb, wa);
        if (j + 2 >= r1) break;
        row(j + 2, Uc_, Ud, Ua, Ub, bc, bd, ba, bb, Db, Dc, Dd, sya, syb, Hya, Hyb, vGXa, vGYa, vGXb, vGYb, wa, wb);
        if (j + 3 >= r1) break;
        row(j + 3, Ud, Ua, Ub, Uc_, bd, ba, bb, bc, Dc, Dd, Da, syb, sya, Hyb, Hya, vGXb, vGYb, vGXa, vGYa, wb, wa);
    }

    // ---- wavefront reductions (fixed butterfly => deterministic in lane 0)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        amx = fmax(amx, __shfl_xor(amx, off, 64));
        amy = fmax(amy, __shfl_xor(amy, off, 64));
        clamps += __shfl_xor(clamps, off, 64);
        bad |= __shfl_xor(bad, off, 64);
    }
    return WavePart{(double)amx, (double)amy, (double)clamps, (double)bad};
}

template <typename T, int STAGE, bool GH, bool CU, bool EP = false, bool BUF = false, bool WB = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(tiled_wpe<T, STAGE, EP, WB>())))
k_stage_tiled(KParams P, const T* __restrict__ Uin, const T* Un, T* Uout, const T* __restrict__ b,
              const T* __restrict__ mu, DevScalars* __restrict__ S, double* __restrict__ bpart,
              double* __restrict__ wpart, int nmax, int R, int nstrips, int nrb)
{
    // XCD-aware block order: consecutive block ids land on different XCDs, so
    // give each XCD a contiguous range of waves (neighbouring strips share halo
    // columns in that XCD's L2).
    const int nblk = gridDim.x;
    int bid = blockIdx.x;
    const int nfull = (nblk / 8) * 8;
    if (bid < nfull) bid = (bid % 8) * (nfull / 8) + bid / 8;
    const int lane = threadIdx.x & 63;
    // wavefront-uniform by construction; readfirstlane lets the compiler keep
    // the strip, row bounds and loop control in scalar registers
    const int w = threadIdx.x >> 6;
    const int wid = __builtin_amdgcn_readfirstlane(bid * 4 + w);
    const int strip = wid % nstrips, rb = wid / nstrips;
    WavePart r{0.0, 0.0, 0.0, 0.0};  // neutral: speeds are >= 0
    if (rb < nrb)  // whole wavefront
        r = stage_tiled_wave<T, STAGE, GH, CU, EP, BUF, WB>(P, Uin, Un, Uout, b, mu, S, bpart, nmax, R, nstrips, nrb,
                                                           strip, rb, lane);
    // one partial record per workgroup (its four wavefronts in order), so
    // the finalize reads a quarter as many (the barrier costs small grids
    // about 0.4 us per stage).  Plain stores: accumulating them with
    // device-wide atomics on one address made the stage 10 % slower.
    __shared__ WavePart wsh[4];
    if (lane == 0) wsh[w] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        WavePart a = wsh[0];
        for (int q = 1; q < 4; q++) {
            a.ax = fmax(a.ax, wsh[q].ax);
            a.ay = fmax(a.ay, wsh[q].ay);
            a.cl += wsh[q].cl;
            a.bd = fmax(a.bd, wsh[q].bd);
        }
        double* wp = wpart + ((size_t)stage_slot(STAGE) * nblk + bid) * 4;
        wp[0] = a.ax;
        wp[1] = a.ay;
        wp[2] = a.cl;
        wp[3] = a.bd;
    }
}

// One work item (scenario, strip, row block) of a batched stage; its partial
// record goes to wave slot `local` of the scenario.  BUF: raw buffer accesses
// (every member's state and DEM below 2 GiB).
template <typename T, int STAGE, bool BUF>
__device__ __forceinline__ void batch_item(const ScenDesc<T>* __restrict__ scen, int item, int R, int lane)
{
    const int sc = item >> 20, local = item & 0xfffff;
    const ScenDesc<T>& D = scen[sc];
    const int strip = local % D.nstrips, rb = local / D.nstrips;
    const WavePart r =
        STAGE == 1 ? stage_tiled_wave<T, 1, false, false, false, BUF>(D.P, D.U, D.U, D.Us, D.b, D.mu, D.S, D.bpart,
                                                                     D.nmax, R, D.nstrips, D.nrb, strip, rb, lane)
                   : stage_tiled_wave<T, 2, false, false, false, BUF>(D.P, D.Us, D.U, D.U, D.b, D.mu, D.S, D.bpart,
                                                                     D.nmax, R, D.nstrips, D.nrb, strip, rb, lane);
    if (lane == 0) {
        double* wp = D.wpart + ((size_t)stage_slot(STAGE) * D.nstrips * D.nrb + local) * 4;
        wp[0] = r.ax;
        wp[1] = r.ay;
        wp[2] = r.cl;
        wp[3] = r.bd;
    }
}

// Batched stage over the work list (every scenario keeps its own time step
// and partial slots, so results equal single-scenario runs; ensemble
// scenarios are Mode-I releases).  Persistent form: a fixed grid of
// wavefronts walks the list with a grid stride.
template <typename T, int STAGE, bool BUF>
__global__ void __launch_bounds__(256)
k_stage_batch(const ScenDesc<T>* __restrict__ scen, const int* __restrict__ work, int nwork, int R)
{
    const int nblk = gridDim.x;
    int bid = blockIdx.x;
    const int nfull = (nblk / 8) * 8;
    if (bid < nfull) bid = (bid % 8) * (nfull / 8) + bid / 8;
    const int lane = threadIdx.x & 63;
    const int nwaves = nblk * 4;
    const int w0 = __builtin_amdgcn_readfirstlane(bid * 4 + (int)(threadIdx.x >> 6));
    for (int w = w0; w < nwork; w += nwaves)
        batch_item<T, STAGE, BUF>(scen, __builtin_amdgcn_readfirstlane(work[w]), R, lane);
}

// Flat form, one wavefront per work item (a grid covering the list): without
// the walk's loop state the FP32 stage-1 body fits the single-scenario
// kernels' occupancy; stage 2 (which reads the scenario's descriptor besides)
// spilled 9 VGPRs at three waves per SIMD and runs 2 % faster per ensemble
// step at two, without spills.
template <typename T, int STAGE, bool BUF>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(STAGE == 1 ? tiled_wpe<T, STAGE>() : (sizeof(T) == 4 ? 2 : 1))))
k_stage_batch_flat(const ScenDesc<T>* __restrict__ scen, const int* __restrict__ work, int nwork, int R)
{
    const int nblk = gridDim.x;
    int bid = blockIdx.x;
    const int nfull = (nblk / 8) * 8;
    if (bid < nfull) bid = (bid % 8) * (nfull / 8) + bid / 8;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(bid * 4 + (int)(threadIdx.x >> 6));
    if (w < nwork) batch_item<T, STAGE, BUF>(scen, __builtin_amdgcn_readfirstlane(work[w]), R, lane);
}

template <typename T>
__global__ void __launch_bounds__(kFinThreads) k_finalize_batch(const ScenDesc<T>* __restrict__ scen, int mode)
{
    const ScenDesc<T>& D = scen[blockIdx.x];
    __shared__ double red[kFinVals];
    fin_reduce<kFinThreads>(D.P, mode, D.wpart,
                            mode == 1 ? D.nw_ref : D.nstrips * D.nrb, red);
    fin_tail_staged(D.P, D.S, red, D.tables, mode);
    if (mode == 0)
        for (int q = threadIdx.x; q < 4 * D.nmax; q += kFinThreads) outflow_accumulate(D.P, D.bpart, D.nmax, q);
}

}  // namespace m2p
