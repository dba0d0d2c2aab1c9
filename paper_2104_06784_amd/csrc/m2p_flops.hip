// m2p_flops.hip -- algorithmic floating-point work of one cell in one stage of
// the forward step, for the roofline of the stage kernels.
//
// The per-cell arithmetic of the fused stage kernel is evaluated once on the
// host with an operation-counting number type, through the same templated
// device functions the kernels call (geometry, dsg, minmod, central_flux,
// sources, visc_*face_c, update_cell, side_speed).  One cell's share is what
// one lane does in one row of the column march: its own geometry and row
// quantities, one x-face and one y-face flux (each face belongs to one cell),
// one new neighbour difference per direction and field (the other one is the
// neighbour's), the sources, the viscous face terms, the update and, in
// stage 2, the Heun average and the CFL speeds (cell_speeds).  Shuffles, loads, stores,
// index arithmetic and the FP64 partial sums are not floating-point work of
// the scheme and are not counted.  The values describe a wet, sliding cell,
// so the Coulomb clamp takes its longer branch.  The formulas are counted in
// the folded forms the FP32 kernels evaluate.
#include <cmath>

#include "m2p.h"
#include "m2p_device.h"

namespace m2p {
namespace {

struct Tally {
    double add, mul, div, sqrt, cmp;
};
Tally g_tally;

// A double that counts the operations applied to it.  Negation and fabs are
// free operand modifiers on CDNA and are not counted.
struct Cnt {
    double v;
    Cnt() : v(0) {}
    Cnt(double x) : v(x) {}
    Cnt operator-() const { return Cnt(-v); }
    Cnt& operator+=(const Cnt& b)
    {
        g_tally.add++;
        v += b.v;
        return *this;
    }
};
inline Cnt operator+(Cnt a, Cnt b) { g_tally.add++; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { g_tally.add++; return Cnt(a.v - b.v); }
// A product with the constant 1 is no operation: it is the earth-pressure
// coefficient of the paper's model, a literal 1 the kernels' compiler removes.
inline Cnt operator*(Cnt a, Cnt b)
{
    if (a.v != 1.0 && b.v != 1.0) g_tally.mul++;
    return Cnt(a.v * b.v);
}
inline Cnt operator/(Cnt a, Cnt b) { g_tally.div++; return Cnt(a.v / b.v); }
inline bool operator<(Cnt a, Cnt b) { g_tally.cmp++; return a.v < b.v; }
inline bool operator>(Cnt a, Cnt b) { g_tally.cmp++; return a.v > b.v; }
inline bool operator<=(Cnt a, Cnt b) { g_tally.cmp++; return a.v <= b.v; }
inline bool operator>=(Cnt a, Cnt b) { g_tally.cmp++; return a.v >= b.v; }
inline Cnt sqrt(Cnt a) { g_tally.sqrt++; return Cnt(std::sqrt(a.v)); }
inline Cnt fabs(Cnt a) { return Cnt(std::fabs(a.v)); }
inline Cnt fmax(Cnt a, Cnt b) { g_tally.cmp++; return Cnt(a.v > b.v ? a.v : b.v); }

}  // namespace

// The count describes the FP32 kernels, which evaluate the folded forms.
template <>
struct Folded<Cnt> : std::true_type {};

namespace {

// Row quantities of the column march (the RowD of the fused kernel).
struct Row {
    Geo<Cnt> g;
    Cnt u, w, cdxu, cdxw, Jh, Gf;
};

// A wet, moving state with non-zero gradients; k selects a neighbour.
void state_of(int k, Cnt u[NF])
{
    const double s = 1.0 + 0.01 * k;
    u[0] = 2.0e-3 * s;
    u[1] = 1.5e-3 * s;
    u[2] = -0.7e-3 * s;
    u[3] = 1.0e-3 * s;
    u[4] = 0.9e-3 * s;
    u[5] = 0.4e-3 * s;
}

// Row quantities of one cell: geometry from the DEM neighbours, the fluid
// velocities and their x central differences, J_b h, J_b h pbar^f.  The x
// neighbours' velocities arrive by shuffle; their values are stand-ins.
Row make_row(const Consts<Cnt>& K, const Cnt u[NF], int k)
{
    Row r;
    const Cnt bE = 0.011 + 0.001 * k, bW = 0.010, bN = 0.012, bS = 0.0105;
    r.g = geometry(bE, bW, bN, bS, K.two_dxi, K.two_deta);
    dsg2(u[4], u[5], u[3], K.md, r.u, r.w);
    r.cdxu = cdiff(Cnt(r.u.v * 1.01), Cnt(r.u.v * 0.99), K.dxi);
    r.cdxw = cdiff(Cnt(r.w.v * 1.01), Cnt(r.w.v * 0.99), K.dxi);
    r.Jh = u[0] + u[3];
    r.Gf = fluid_G(u[0], u[3], r.g);
    return r;
}

// One cell's share of one stage (see the file header).
template <bool H2>
void cell_stage_t(const Consts<Cnt>& K, int stage, bool visc, int flags)
{
    Tally saved = g_tally;
    // values that earlier rows / neighbouring lanes provide (not counted)
    Cnt Uc[NF], Un1[NF], U2[NF], UW[NF], unr[NF];
    state_of(0, Uc);
    state_of(1, Un1);
    state_of(2, U2);
    state_of(3, UW);
    state_of(4, unr);
    Row Dm = make_row(K, UW, 0), D0 = make_row(K, Uc, 1);
    Cnt sy0[NF], dyprev[NF], dxW[NF], Hy[NF], HxL[NF];
    for (int k = 0; k < NF; k++) {
        dyprev[k] = Un1[k].v - Uc[k].v;
        dxW[k] = Uc[k].v - UW[k].v;
        sy0[k] = 0.5 * dxW[k].v;
        Hy[k] = 1e-4 * (k + 1);
        HxL[k] = 1.1e-4 * (k + 1);
    }
    Cnt vGX = 1e-6, vGY = -1e-6;
    g_tally = saved;

    // ---- counted: row j+1 quantities, y-slopes, y-face j+1/2
    Row D1 = make_row(K, Un1, 2);
    Cnt sy1[NF], uL[NF], uR[NF];
    for (int k = 0; k < NF; k++) {
        const Cnt dn1 = U2[k] - Un1[k];
        sy1[k] = minmod(dyprev[k], dn1);
        uL[k] = Uc[k] + Cnt(0.5) * sy0[k];
        uR[k] = Un1[k] - Cnt(0.5) * sy1[k];
    }
    Cnt HyN[NF];
    central_flux<Cnt, H2>(K, uL, D0.g, uR, D1.g, 1, HyN);
    Cnt vGXN = 0.0, vGYN = 0.0;
    if (visc)
        visc_yface_c(D0.u, D0.w, D1.u, D1.w, D0.cdxu, D0.cdxw, D1.cdxu, D1.cdxw, D0.Jh, D1.Jh, D0.g, D1.g, K.deta,
                     vGXN, vGYN);
    // ---- x-face i+1/2: slopes of this cell, right value of the east cell
    Cnt um[NF], upR[NF], Hx[NF];
    for (int k = 0; k < NF; k++) {
        const Cnt dE = Cnt(Uc[k].v * 1.02) - Uc[k];
        const Cnt sx = minmod(dxW[k], dE);
        um[k] = Uc[k] + Cnt(0.5) * sx;
        const Cnt up = Uc[k] - Cnt(0.5) * sx;  // right value of face i-1/2, sent west
        upR[k] = up.v * 1.01;
    }
    central_flux<Cnt, H2>(K, um, D0.g, upR, D1.g, 0, Hx);
    // ---- sources
    Cnt dn[6];
    dn[0] = (Cnt(D0.g.nX.v * 1.01) - Cnt(D0.g.nX.v * 0.99)) / K.two_dxi;
    dn[1] = (Cnt(D0.g.nY.v * 1.01) - Cnt(D0.g.nY.v * 0.99)) / K.two_dxi;
    dn[2] = (Cnt(D0.g.nZ.v * 1.01) - Cnt(D0.g.nZ.v * 0.99)) / K.two_dxi;
    dn[3] = (D1.g.nX - Dm.g.nX) / K.two_deta;
    dn[4] = (D1.g.nY - Dm.g.nY) / K.two_deta;
    dn[5] = (D1.g.nZ - Dm.g.nZ) / K.two_deta;
    const Cnt dGx = (Cnt(D0.Gf.v * 1.01) - Cnt(D0.Gf.v * 0.99)) / K.two_dxi;
    const Cnt dGy = (D1.Gf - Dm.Gf) / K.two_deta;
    Src<Cnt> Sr;
    sources(K, flags, Uc, D0.g, dn, dGx, dGy, Sr);
    Cnt svx = 0.0, svy = 0.0;
    if (visc) {
        const Cnt cdyu = cdiff(D1.u, Dm.u, K.deta);
        const Cnt cdyw = cdiff(D1.w, Dm.w, K.deta);
        Cnt FX1, FY1;
        visc_xface_c(D0.u, D0.w, Cnt(D0.u.v * 1.01), Cnt(D0.w.v * 1.01), cdyu, cdyw, Cnt(cdyu.v * 1.01),
                     Cnt(cdyw.v * 1.01), D0.Jh, Cnt(D0.Jh.v * 1.01), D0.g, D1.g, K.dxi, FX1, FY1);
        const Cnt FX0 = FX1.v * 0.99, FY0 = FY1.v * 0.99;
        const Cnt SvX = (FX1 - FX0) / K.dxi + (vGXN - vGX) / K.deta;
        const Cnt SvY = (FY1 - FY0) / K.dxi + (vGYN - vGY) / K.deta;
        svx = K.eps * Sr.phif * K.inv_n_r * SvX;
        svy = K.eps * Sr.phif * K.inv_n_r * SvY;
    }
    // ---- update (a sliding cell: the clamp takes its longer branch)
    Cnt out[NF];
    const Cnt dt = 1e-3, tmu = 0.05;
    update_cell<Cnt, H2>(K, Uc, D0.g, HxL, Hx, Hy, HyN, Sr, svx, svy, dt, tmu, out);
    if (stage == 2) {
        for (int k = 0; k < NF; k++) out[k] = Cnt(0.5) * (unr[k] + out[k]);
        Cnt sx, sy, amx = 0.0, amy = 0.0;
        cell_speeds(K, out, D0.g, sx, sy);
        amx = fmax(amx, sx);
        amy = fmax(amy, sy);
    }
}

// Stage 1 carries face fluxes as 2 H (the FP32 stage-1 kernel's form).
void cell_stage(const Consts<Cnt>& K, int stage, bool visc, int flags)
{
    if (stage == 1)
        cell_stage_t<true>(K, stage, visc, flags);
    else
        cell_stage_t<false>(K, stage, visc, flags);
}

KParams count_params(int visc)
{
    KParams P{};
    P.dxi = P.deta = 0.01;
    P.two_dxi = P.two_deta = 0.02;
    P.eps = 0.01;
    P.alpha = 0.37;
    P.one_m_alpha = 0.63;
    P.md = 1e-7;
    P.eps_chi = 0.0;
    P.tan_d = std::tan(20.0 * M_PI / 180.0);
    P.c_d = 6.0;
    P.inv_n_r = visc ? 1.0 / 268.0 : 0.0;
    P.theta_b = 5.0;
    P.visc = visc;
    return P;
}

}  // namespace
}  // namespace m2p

extern "C" int m2p_stage_flops(int32_t stage, int32_t visc, double* out)
{
    using namespace m2p;
    if ((stage != 1 && stage != 2) || out == nullptr) return M2P_EINVAL;
    const KParams P = count_params(visc != 0);
    const Consts<Cnt> K(P);
    g_tally = Tally{0, 0, 0, 0, 0};
    cell_stage(K, stage, visc != 0, 0);
    out[0] = g_tally.add;
    out[1] = g_tally.mul;
    out[2] = g_tally.div;
    out[3] = g_tally.sqrt;
    out[4] = g_tally.cmp;
    return M2P_OK;
}
