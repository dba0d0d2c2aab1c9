// m2p_device.h -- device arithmetic of one forward-Euler stage of the
// two-phase depth-integrated shallow-flow model (Appendix A of the paper)
// with the central scheme of Sect. 2.2.  Templated on the state type T
// (float or double).  The FP64 build is compiled without FMA contraction and
// follows the evaluation order written here exactly; the FP32 build uses fast
// reciprocals and fuses multiply-adds within each expression, and across
// statements only in the functions a stage evaluates once per cell (the
// "fp contract(fast)" blocks), so that a quantity a tile recomputes at its
// edge has the same bits as in the neighbouring tile.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <type_traits>

// Host-and-device so that the arithmetic can also be evaluated on the host
// with other number types (operation counting).
#define M2P_FN __host__ __device__ __forceinline__

namespace m2p {

constexpr int NF = 6;        // m^s, p^s_X, p^s_Y, m^f, p^f_X, p^f_Y
constexpr int MAX_SEG = 8;   // Mode-II inflow segments
constexpr int BOFF = 64;     // column offset of cell 0 in the padded DEM rows
constexpr int BHALO = 2;     // ghost rows / columns of the padded DEM

struct SegDesc {
    int side, i0, ncells, nt, toff;
};

// Constants of a scenario, all dimensionless.  Passed by value to kernels.
struct KParams {
    int nx, ny, pitch, bpitch;
    int bc[4];
    int flags, has_mu, nseg, visc;
    double dxi, deta, two_dxi, two_deta;
    double eps, alpha, one_m_alpha, md, eps_chi, tan_d;
    double c_d, inv_n_r, theta_b;
    double T, V, H, L, dx, dy, cfl, a_floor, dt_floor;
    SegDesc seg[MAX_SEG];   // Mode-II segments with a discharge hydrograph (face flux)
    int nsseg;
    int rk;                 // stages per step: 2 (Heun) or 3 (SSP Runge-Kutta)
    SegDesc sseg[MAX_SEG];  // Mode-II segments with a state hydrograph (ghost cells)
    int ntab;               // doubles in the hydrograph table of both kinds of segment
    double cos2_int;        // cos^2 of the internal friction angle (earth-pressure option)
    double v_eps;           // regularisation speed of the smooth-friction option, / sqrt(g L)
};

// Scalars that live on the device across steps (time, dt, reductions).
struct DevScalars {
    double t, dt, dt_last, t_end;
    double in_s, in_f, out_s, out_f;
    long long steps;
    unsigned long long clamps;
    unsigned int status;
    unsigned int pad;
    double inflow[3][MAX_SEG][4];      // per stage: q, m_in, v_in, phi
    double sghost[3][MAX_SEG][NF];     // per stage: ghost state of each state segment
    const double* dt_sched;            // optional prescribed (frozen) time steps, dimensionless
    long long n_sched;
    double* dt_log;                    // optional record: the finalize stores the next step's dt at
    long long log_base, n_log;         //   dt_log[steps - log_base] when that index is in [0, n_log)
};

// Boundary outflow integrals, [4 sides][nmax][2 phases] doubles: each step
// adds, per boundary face and stage in stage order, the stage's quadrature
// weight times dt times its volume flux through the face to that face's
// running integral (Heun: dt/2, dt/2; the three-stage method: dt/6, dt/6,
// 2 dt/3).  The stages store their fluxes in slots and the finalize adds them
// (one thread per face), so each integral is a fixed-order sum; they are
// summed over the faces on demand.
constexpr double stage_weight(int kind, int rk)
{
    return kind == 1 ? (rk == 3 ? 1.0 / 6.0 : 0.5) : (kind == 2 ? 0.5 : (kind == 3 ? 1.0 / 6.0 : 2.0 / 3.0));
}

// Stage kinds of a step.  Heun, the paper's two-step modified Euler method:
// kinds 1 then 2.  Three-stage SSP Runge-Kutta: kinds 1, 3, 4.
//   1: U1 = E(U^n)   2: (U^n + E(U1)) / 2   3: 3/4 U^n + 1/4 E(U1)
//   4: 1/3 U^n + 2/3 E(U2)
// The slot is the stage's index within the step (its time, inflow states and
// partial sums); kinds 2 and 4 end the step and give the CFL speeds.
constexpr int stage_slot(int kind) { return kind == 1 ? 0 : (kind == 4 ? 2 : 1); }
constexpr bool stage_last(int kind) { return kind == 2 || kind == 4; }

template <int KIND, typename T>
M2P_FN T stage_combine(T un, T e)
{
    if constexpr (KIND == 2) return T(0.5) * (un + e);
    else if constexpr (KIND == 3) return T(0.75) * un + T(0.25) * e;
    else return T(1.0 / 3.0) * un + T(2.0 / 3.0) * e;
}

template <typename T>
struct Geo {
    T bX, bY, J, c, nX, nY, nZ, A11, A12, A21, A22;
};

// The FP32 build evaluates some formulas in algebraically folded forms with
// fewer operations: J_b c = 1 (c = n_Z = 1/J_b), so h^s = m^s c and
// eps J_b h A N^s = eps (1 - alpha)/2 h h^s A; products of constants are
// folded.  The FP64 build (bitwise parity with the FP64 oracle) and the
// dual-number adjoint evaluate the formulas as written.
template <typename T>
struct Folded : std::false_type {};
template <>
struct Folded<float> : std::true_type {};

// minmod(a, b): the argument of smaller magnitude when both have the same
// strict sign, else 0 (written with selects so the compiler emits no branch).
// That is exactly the median of (a, b, 0), one v_med3_f32 in FP32.
template <typename T>
M2P_FN T minmod(T a, T b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (std::is_same<T, float>::value) return __builtin_amdgcn_fmed3f(a, b, 0.0f);
#endif
    const T lo = a < b ? a : b, hi = a > b ? a : b;
    const bool pos = (int)(a > T(0)) & (int)(b > T(0));
    const bool neg = (int)(a < T(0)) & (int)(b < T(0));
    return pos ? lo : (neg ? hi : T(0));
}

// max of two values for the FP32 forms: one v_max_f32 (the same value as
// the select a > b ? a : b for the finite, non-negative operands it gets)
M2P_FN float fmax_f(float a, float b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_fmaxf(a, b);
#else
    return a > b ? a : b;
#endif
}
template <typename T>
M2P_FN T fmax_f(T a, T b)
{
    return a > b ? a : b;
}

// Continuous desingularisation of num / den (Kurganov-Petrova 2007):
// 2 den num / (den^2 + max(den^2, md^2)).
template <typename T>
M2P_FN T dsg(T num, T den, T md)
{
    if constexpr (Folded<T>::value) {
        const T d2 = den * den;
        return ((den + den) * num) / (d2 + fmax_f(d2, md * md));
    }
    T d2 = den * den;
    T m2 = md * md;
    return (T(2) * den * num) / (d2 + (d2 > m2 ? d2 : m2));
}

// Both ratios n1 / den and n2 / den, desingularised as dsg does.  The FP32
// build computes the common factor 2 den / (den^2 + max(den^2, md^2)) once
// (one multiplication per ratio instead of two).
template <typename T>
M2P_FN void dsg2(T n1, T n2, T den, T md, T& v1, T& v2)
{
    if constexpr (Folded<T>::value) {
        const T d2 = den * den;
        const T m2 = md * md;
        const T sc = (den + den) / (d2 + fmax_f(d2, m2));
        v1 = n1 * sc;
        v2 = n2 * sc;
        return;
    }
    v1 = dsg(n1, den, md);
    v2 = dsg(n2, den, md);
}

// 1 / sqrt(x): one hardware reciprocal square root in FP32 device code.
template <typename T>
M2P_FN T rsq(T x)
{
    return T(1) / sqrt(x);
}
M2P_FN float rsq(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsqf(x);
#else
    return 1.0f / std::sqrt(x);
#endif
}

// Basal geometry from the four DEM neighbours (b / L): tangents
// (1, 0, b_X), (0, 1, b_Y), unit normal (-b_X, -b_Y, 1)/s, J_b = s, c = n_Z,
// A = inverse surface metric.
template <typename T>
M2P_FN Geo<T> geometry(T bE, T bW, T bN, T bS, T two_dxi, T two_deta)
{
    Geo<T> g;
    T bX = (bE - bW) / two_dxi;
    T bY = (bN - bS) / two_deta;
    if constexpr (Folded<T>::value) {
        const T q = T(1) + bX * bX + bY * bY;
        const T c = rsq(q), c2 = c * c;
        g.bX = bX;
        g.bY = bY;
        g.J = q * c;
        g.c = c;
        g.nX = -bX * c;
        g.nY = -bY * c;
        g.nZ = c;
        g.A11 = (T(1) + bY * bY) * c2;
        g.A12 = -bX * bY * c2;
        g.A21 = g.A12;
        g.A22 = (T(1) + bX * bX) * c2;
        return g;
    }
    T s = sqrt(T(1) + bX * bX + bY * bY);
    g.bX = bX;
    g.bY = bY;
    g.J = s;
    g.c = T(1) / s;
    g.nX = -bX / s;
    g.nY = -bY / s;
    g.nZ = T(1) / s;
    g.A11 = (T(1) + bY * bY) / (s * s);
    g.A12 = -bX * bY / (s * s);
    g.A21 = g.A12;
    g.A22 = (T(1) + bX * bX) / (s * s);
    return g;
}

template <typename T>
struct Consts {
    T eps, al, oma, md, eps_chi, tan_d, c_d, inv_n_r, theta_b;
    T dxi, deta, two_dxi, two_deta;
    // folded constants of the FP32 forms: eps (1 - alpha) / 2, eps / 2,
    // (1 - alpha) / 2, -eps alpha, theta_b / (N_R eps), 1 / (2 dxi), 1 / (2 deta),
    // 1 / dxi, 1 / deta
    T k_ps, k_pf, half_oma, m_eps_al, k_fr, half_rdxi, half_rdeta, rdxi, rdeta;
    // smooth-friction option (flags bit 4) and its regularisation speed
    bool smooth;
    T veps;
    M2P_FN explicit Consts(const KParams& P)
        : eps(T(P.eps)), al(T(P.alpha)), oma(T(P.one_m_alpha)), md(T(P.md)), eps_chi(T(P.eps_chi)),
          tan_d(T(P.tan_d)), c_d(T(P.c_d)), inv_n_r(T(P.inv_n_r)), theta_b(T(P.theta_b)),
          dxi(T(P.dxi)), deta(T(P.deta)), two_dxi(T(P.two_dxi)), two_deta(T(P.two_deta)),
          k_ps(T(P.eps * (1.0 - P.alpha) / 2.0)), k_pf(T(P.eps / 2.0)), half_oma(T((1.0 - P.alpha) / 2.0)),
          m_eps_al(T(-P.eps * P.alpha)), k_fr(T(P.theta_b * P.inv_n_r / P.eps)), half_rdxi(T(0.5 / P.dxi)),
          half_rdeta(T(0.5 / P.deta)), rdxi(T(1.0 / P.dxi)), rdeta(T(1.0 / P.deta)),
          smooth((P.flags & 16) != 0), veps(T(P.v_eps)) {}  // 16: M2P_F_SMOOTH_FRICTION
};


// Physical flux of one reconstructed side of a face (flux vectors F, G of
// Appendix A with the owner cell's geometry), the conserved values entering
// the numerical diffusion and the phase speeds |v_n| + sqrt(dP/dm); with OS
// (one-sided), a = v_n + sqrt(dP/dm) and am = v_n - sqrt(dP/dm) instead.
template <typename T, bool OS = false>
M2P_FN void side_flux(const Consts<T>& K, const T u[NF], const Geo<T>& g, int d,
                                          T F[NF], T qv[NF], T a[2], T* am = nullptr, T kep = T(1))
{
    if constexpr (Folded<T>::value) {
        const T ms = u[0], mf = u[3];
        const T hs = ms * g.c, hf = mf * g.c, h = hs + hf;
        T vXs, vYs, vXf, vYf;
        dsg2(u[1], u[2], ms, K.md, vXs, vYs);
        dsg2(u[4], u[5], mf, K.md, vXf, vYf);
        const T Ax = d == 0 ? g.A11 : g.A21;
        const T Ay = d == 0 ? g.A12 : g.A22;
        const T Ann = d == 0 ? g.A11 : g.A22;
        const T vns = d == 0 ? vXs : vYs;
        const T vnf = d == 0 ? vXf : vYf;
        const T Ps = kep * (K.k_ps * h * hs);  // eps J_b h N^s / c, times the earth-pressure coefficient
        const T Pf = K.k_pf * h * h;   // eps J_b h pbar^f / c
        qv[0] = ms;
        qv[1] = ms * vXs;
        qv[2] = ms * vYs;
        qv[3] = mf;
        qv[4] = mf * vXf;
        qv[5] = mf * vYf;
        F[0] = ms * vns;
        F[1] = qv[1] * vns + Ps * Ax;
        F[2] = qv[2] * vns + Ps * Ay;
        F[3] = mf * vnf;
        F[4] = qv[4] * vnf + Pf * Ax;
        F[5] = qv[5] * vnf + Pf * Ay;
        const T ac = K.eps * Ann * g.c;
        const T cs = kep * (ac * K.half_oma * (h + hs));
        const T cf = ac * h;
        const T rs = sqrt(cs > T(0) ? cs : T(0)), rf = sqrt(cf > T(0) ? cf : T(0));
        if constexpr (OS) {
            a[0] = vns + rs;
            am[0] = vns - rs;
            a[1] = vnf + rf;
            am[1] = vnf - rf;
        } else {
            a[0] = fabs(vns) + rs;
            a[1] = fabs(vnf) + rf;
        }
        return;
    }
    T ms = u[0], mf = u[3];
    T hs = ms / g.J, hf = mf / g.J, h = hs + hf;
    T vXs = dsg(u[1], ms, K.md), vYs = dsg(u[2], ms, K.md);
    T vXf = dsg(u[4], mf, K.md), vYf = dsg(u[5], mf, K.md);
    T Ns = kep * (g.c * (T(1) - K.al) * hs / T(2));  // times the earth-pressure coefficient
    T pf = g.c * h / T(2);
    T Ax = d == 0 ? g.A11 : g.A21;
    T Ay = d == 0 ? g.A12 : g.A22;
    T Ann = d == 0 ? g.A11 : g.A22;
    T vns = d == 0 ? vXs : vYs;
    T vnf = d == 0 ? vXf : vYf;
    F[0] = ms * vns;
    F[1] = ms * vXs * vns + K.eps * g.J * h * Ax * Ns;
    F[2] = ms * vYs * vns + K.eps * g.J * h * Ay * Ns;
    F[3] = mf * vnf;
    F[4] = mf * vXf * vnf + K.eps * g.J * h * Ax * pf;
    F[5] = mf * vYf * vnf + K.eps * g.J * h * Ay * pf;
    qv[0] = ms;
    qv[1] = ms * vXs;
    qv[2] = ms * vYs;
    qv[3] = mf;
    qv[4] = mf * vXf;
    qv[5] = mf * vYf;
    T cs = kep * (K.eps * Ann * g.c * (T(1) - K.al) * (h + hs) / T(2));
    T cf = K.eps * Ann * g.c * h;
    T rs = sqrt(cs > T(0) ? cs : T(0)), rf = sqrt(cf > T(0) ? cf : T(0));
    if constexpr (OS) {
        a[0] = vns + rs;
        am[0] = vns - rs;
        a[1] = vnf + rf;
        am[1] = vnf - rf;
    } else {
        a[0] = fabs(vns) + rs;
        a[1] = fabs(vnf) + rf;
    }
}

// Phase speeds only (identical arithmetic to side_flux).
template <typename T>
M2P_FN void side_speed(const Consts<T>& K, const T u[NF], const Geo<T>& g, int d, T a[2], T kep = T(1))
{
    if constexpr (Folded<T>::value) {
        const T ms = u[0], mf = u[3];
        const T hs = ms * g.c, hf = mf * g.c, h = hs + hf;
        const T vns = d == 0 ? dsg(u[1], ms, K.md) : dsg(u[2], ms, K.md);
        const T vnf = d == 0 ? dsg(u[4], mf, K.md) : dsg(u[5], mf, K.md);
        const T ac = K.eps * (d == 0 ? g.A11 : g.A22) * g.c;
        const T cs = kep * (ac * K.half_oma * (h + hs));
        const T cf = ac * h;
        a[0] = fabs(vns) + sqrt(cs > T(0) ? cs : T(0));
        a[1] = fabs(vnf) + sqrt(cf > T(0) ? cf : T(0));
        return;
    }
    T ms = u[0], mf = u[3];
    T hs = ms / g.J, hf = mf / g.J, h = hs + hf;
    T vns = d == 0 ? dsg(u[1], ms, K.md) : dsg(u[2], ms, K.md);
    T vnf = d == 0 ? dsg(u[4], mf, K.md) : dsg(u[5], mf, K.md);
    T Ann = d == 0 ? g.A11 : g.A22;
    T cs = kep * (K.eps * Ann * g.c * (T(1) - K.al) * (h + hs) / T(2));
    T cf = K.eps * Ann * g.c * h;
    a[0] = fabs(vns) + sqrt(cs > T(0) ? cs : T(0));
    a[1] = fabs(vnf) + sqrt(cf > T(0) ? cf : T(0));
}

// CFL speeds of a cell in both directions, each the maximum over the phases
// of side_speed.  The FP32 forms compute the velocity ratios in pairs (one
// desingularisation factor per phase); otherwise side_speed twice.
template <typename T>
M2P_FN void cell_speeds(const Consts<T>& K, const T u[NF], const Geo<T>& g, T& ax, T& ay, T kep = T(1))
{
    if constexpr (Folded<T>::value) {
        _Pragma("clang fp contract(fast)")
        const T ms = u[0], mf = u[3];
        const T hs = ms * g.c, hf = mf * g.c, h = hs + hf;
        T vXs, vYs, vXf, vYf;
        dsg2(u[1], u[2], ms, K.md, vXs, vYs);
        dsg2(u[4], u[5], mf, K.md, vXf, vYf);
        const T hhs = kep * (K.half_oma * (h + hs));
        const T acx = K.eps * g.A11 * g.c, acy = K.eps * g.A22 * g.c;
        const T csx = acx * hhs, cfx = acx * h, csy = acy * hhs, cfy = acy * h;
        const T axs = fabs(vXs) + sqrt(csx > T(0) ? csx : T(0)), axf = fabs(vXf) + sqrt(cfx > T(0) ? cfx : T(0));
        const T ays = fabs(vYs) + sqrt(csy > T(0) ? csy : T(0)), ayf = fabs(vYf) + sqrt(cfy > T(0) ? cfy : T(0));
        ax = axs > axf ? axs : axf;
        ay = ays > ayf ? ays : ayf;
        return;
    }
    T a[2];
    side_speed(K, u, g, 0, a, kep);
    ax = a[0] > a[1] ? a[0] : a[1];
    side_speed(K, u, g, 1, a, kep);
    ay = a[0] > a[1] ? a[0] : a[1];
}

// Face fluxes may be carried as twice the flux (H2, FP32 forms only): the
// factor 1/2 is then applied once where a face flux is used (the update,
// the boundary outflow slots) instead of once per component and face.
template <typename T, bool H2>
constexpr bool carry_2h()
{
    return H2 && Folded<T>::value;
}

// Central flux per phase (twice the flux when carried as 2 H).
// Default, Kurganov-Tadmor: (F- + F+)/2 - a/2 (U+ - U-), a the larger of the
// two sides' phase speeds.  CU, central-upwind with one-sided local speeds
// (the form Kurganov-Petrova 2007 builds on): a+ = max(largest speed of the
// two sides, 0), a- = min(smallest speed, 0),
//   H = (a+ F- - a- F+) / (a+ - a-) + a+ a- / (a+ - a-) (U+ - U-),
// and (F- + F+)/2 where a+ = a- = 0 (a dry face).
// dqm (the well-balanced option): the jumps of the two masses in the
// numerical diffusion, in place of m+ - m-.
template <typename T, bool H2 = false, bool CU = false>
M2P_FN void central_flux(const Consts<T>& K, const T uL[NF], const Geo<T>& gL,
                                             const T uR[NF], const Geo<T>& gR, int d, T H[NF], T kL = T(1),
                                             T kR = T(1), const T* dqm = nullptr)
{
    // jump of a conserved field across the face in the numerical diffusion
    auto jump = [&](const T* qL, const T* qR, int k) {
        return (dqm && k % 3 == 0) ? dqm[k / 3] : qR[k] - qL[k];
    };
    if constexpr (CU) {
        T FL[NF], FR[NF], qL[NF], qR[NF], hiL[2], loL[2], hiR[2], loR[2];
        side_flux<T, true>(K, uL, gL, d, FL, qL, hiL, loL, kL);
        side_flux<T, true>(K, uR, gR, d, FR, qR, hiR, loR, kR);
#pragma unroll
        for (int ph = 0; ph < 2; ph++) {
            T ap = hiL[ph] > hiR[ph] ? hiL[ph] : hiR[ph];
            T am = loL[ph] < loR[ph] ? loL[ph] : loR[ph];
            ap = ap < T(0) ? T(0) : ap;
            am = am > T(0) ? T(0) : am;
            const T den = ap - am;
            const bool wet = den > T(0);
            if constexpr (Folded<T>::value) {
                // one reciprocal per phase; the 2 H carry folds into it
                const T r = wet ? (carry_2h<T, H2>() ? T(2) : T(1)) / den : T(0);
                const T c0 = carry_2h<T, H2>() ? T(1) : T(0.5);
#pragma unroll
                for (int k = 3 * ph; k < 3 * ph + 3; k++)
                    H[k] = wet ? (ap * FL[k] - am * FR[k]) * r + ap * am * r * jump(qL, qR, k)
                               : c0 * (FL[k] + FR[k]);
            } else {
#pragma unroll
                for (int k = 3 * ph; k < 3 * ph + 3; k++)
                    H[k] = wet ? (ap * FL[k] - am * FR[k]) / den + ap * am / den * jump(qL, qR, k)
                               : T(0.5) * (FL[k] + FR[k]);
            }
        }
        return;
    }
    T FL[NF], FR[NF], qL[NF], qR[NF], aL[2], aR[2];
    side_flux<T>(K, uL, gL, d, FL, qL, aL, nullptr, kL);
    side_flux<T>(K, uR, gR, d, FR, qR, aR, nullptr, kR);
#pragma unroll
    for (int ph = 0; ph < 2; ph++) {
        T a = aL[ph] > aR[ph] ? aL[ph] : aR[ph];
#pragma unroll
        for (int k = 3 * ph; k < 3 * ph + 3; k++) {
            if constexpr (carry_2h<T, H2>())
                H[k] = (FL[k] + FR[k]) - a * jump(qL, qR, k);
            else
                H[k] = T(0.5) * (FL[k] + FR[k]) - T(0.5) * a * jump(qL, qR, k);
        }
    }
}

// KParams.flags bits of the central-upwind face flux and of the earth-pressure
// coefficients (M2P_F_CENTRAL_UPWIND, M2P_F_EARTH_PRESSURE).
constexpr int kFlagCentralUpwind = 4;
constexpr int kFlagEarthPressure = 8;
constexpr int kFlagSmoothFriction = 16;
constexpr int kFlagWellBalanced = 32;

// The face flux the flags select, chosen at run time (the tiled kernels take
// the choice as a template argument instead); kL, kR: the earth-pressure
// coefficients of the two sides' owner cells in the face's direction.
template <typename T>
M2P_FN void face_flux_sel(const Consts<T>& K, int flags, const T uL[NF], const Geo<T>& gL, const T uR[NF],
                          const Geo<T>& gR, int d, T H[NF], T kL = T(1), T kR = T(1), const T* dqm = nullptr)
{
    if (flags & kFlagCentralUpwind)
        central_flux<T, false, true>(K, uL, gL, uR, gR, d, H, kL, kR, dqm);
    else
        central_flux(K, uL, gL, uR, gR, d, H, kL, kR, dqm);
}

// ------------------------------------- well-balanced option (flags bit 5)
// Hydrostatic reconstruction (Audusse et al. 2004; Sect. 2.2 cites the
// well-balanced central-upwind schemes) in this model's variables.  At rest
// a phase's pressure flux through a face is (1 + b_t^2) eta^2 / (2 eps) (times
// 1 - alpha for the solid) and its basal-pressure source -(eta / eps) b_n, with
// eta = eps c^2 m; on beds that vary in one direction the rest states are
// b + eta = const per phase.  Per cell and direction the face values of eta
// and of the bed come from minmod slopes; at a face B* is the larger bed value,
// eta* = max(0, eta + b - B*) per side, the flux is taken from the starred
// states (m* = eta* / (eps c^2), momenta scaled by m* / m, the masses'
// numerical diffusion on eta* weighted with the larger 1 / (eps c^2) of the
// two sides), and each cell adds the difference of the
// pressure terms of its unstarred and starred face states; the hydrostatic
// part of the basal-pressure source takes the matching discrete form.

// Face values (minus, plus side) of eta and of the bed of the middle cell of
// three along a direction; sbo (if given) receives the bed slope.
template <typename T>
M2P_FN void wb_cell(T e0, T e1, T e2, T b0, T b1, T b2, T& em, T& ep, T& bm, T& bp, T* sbo = nullptr)
{
    const T se = minmod(e1 - e0, e2 - e1);
    const T sb = minmod(b1 - b0, b2 - b1);
    em = e1 - T(0.5) * se;
    ep = e1 + T(0.5) * se;
    bm = b1 - T(0.5) * sb;
    bp = b1 + T(0.5) * sb;
    if (sbo) *sbo = sb;
}

// The difference of a face's two bed values, left minus right, from the two
// cells' beds bl, br and slopes sl, sr: (bl - br) + (sl + sr) / 2, the bed
// difference of neighbouring cells formed first (exact in floating point for
// beds within a factor two of each other), so the FP32 forms keep it to the
// precision of the slopes rather than of the bed elevation.
template <typename T>
M2P_FN T wb_bed_jump(T bl, T br, T sl, T sr)
{
    return (bl - br) + T(0.5) * (sl + sr);
}

// Pressure parts of a side's physical flux (the momentum components of
// side_flux, in the same form).
template <typename T>
M2P_FN void wb_pterm(const Consts<T>& K, const T u[NF], const Geo<T>& g, int d, T P[NF])
{
    const T Ax = d == 0 ? g.A11 : g.A21, Ay = d == 0 ? g.A12 : g.A22;
    P[0] = T(0);
    P[3] = T(0);
    if constexpr (Folded<T>::value) {
        const T hs = u[0] * g.c, hf = u[3] * g.c, h = hs + hf;
        const T Ps = K.k_ps * h * hs, Pf = K.k_pf * h * h;
        P[1] = Ps * Ax;
        P[2] = Ps * Ay;
        P[4] = Pf * Ax;
        P[5] = Pf * Ay;
    } else {
        const T hs = u[0] / g.J, hf = u[3] / g.J, h = hs + hf;
        const T Ns = g.c * (T(1) - K.al) * hs / T(2), pf = g.c * h / T(2);
        P[1] = K.eps * g.J * h * Ax * Ns;
        P[2] = K.eps * g.J * h * Ay * Ns;
        P[4] = K.eps * g.J * h * Ax * pf;
        P[5] = K.eps * g.J * h * Ay * pf;
    }
}

// One face along d between a left and a right cell: uL, uR the plain
// reconstructed states, c2L, c2R the cells' c^2, etaL/bL the left cell's
// plus-side face values (per phase), etaR/bR the right cell's minus-side ones.
// A wall face (wallL: the left cell is the ghost; wallR: the right one) takes
// the ghost side as the mirror image of the edge cell (its face values, c and
// geometry), so no mass crosses the wall.  Out: the flux H and the corrections
// cL, cR of the left and right cell.  The FP32 forms take the bed values'
// difference dB (wb_bed_jump) instead of the face values, eta* as
// max(0, eta + min(0, +-dB)) (the same value; the bed elevation never enters
// a sum with the much smaller eta), and one reciprocal of eps c^2 per side.
template <typename T>
M2P_FN void wb_face(const Consts<T>& K, int flags, const T uL[NF], Geo<T> gL, T c2L, const T uR[NF], Geo<T> gR,
                    T c2R, const T etaL_[2], const T bL_[2], const T etaR_[2], const T bR_[2], T dB, bool wallL,
                    bool wallR, int d, T H[NF], T cL[NF], T cR[NF])
{
    // (the flux of the starred states is the one the flags select)
    if (wallL) {
        gL = gR;
        c2L = c2R;
    }
    if (wallR) {
        gR = gL;
        c2R = c2L;
    }
    T sL[NF], sR[NF], dqm[2];
    if constexpr (Folded<T>::value) {
        const T rL = T(1) / (K.eps * c2L), rR = T(1) / (K.eps * c2R);
        const T wd = rL > rR ? rL : rR;
        const T dBw = (wallL || wallR) ? T(0) : dB;
        const T dL = dBw < T(0) ? dBw : T(0), dR = dBw > T(0) ? -dBw : T(0);
#pragma unroll
        for (int ph = 0; ph < 2; ph++) {
            T etaL = etaL_[ph], etaR = etaR_[ph];
            if (wallL) etaL = etaR;
            if (wallR) etaR = etaL;
            T esL = etaL + dL, esR = etaR + dR;
            if (esL < T(0)) esL = T(0);
            if (esR < T(0)) esR = T(0);
            const int k0 = 3 * ph;
            const T fL = etaL > T(0) ? esL / etaL : T(0), fR = etaR > T(0) ? esR / etaR : T(0);
            sL[k0] = esL * rL;
            sL[k0 + 1] = uL[k0 + 1] * fL;
            sL[k0 + 2] = uL[k0 + 2] * fL;
            sR[k0] = esR * rR;
            sR[k0 + 1] = uR[k0 + 1] * fR;
            sR[k0 + 2] = uR[k0 + 2] * fR;
            dqm[ph] = (esR - esL) * wd;
            cL[k0] = etaL * rL;
            cL[k0 + 1] = uL[k0 + 1];
            cL[k0 + 2] = uL[k0 + 2];
            cR[k0] = etaR * rR;
            cR[k0 + 1] = uR[k0 + 1];
            cR[k0 + 2] = uR[k0 + 2];
        }
    } else {
#pragma unroll
        for (int ph = 0; ph < 2; ph++) {
            T etaL = etaL_[ph], bL = bL_[ph], etaR = etaR_[ph], bR = bR_[ph];
            if (wallL) {
                etaL = etaR;
                bL = bR;
            }
            if (wallR) {
                etaR = etaL;
                bR = bL;
            }
            const T Bs = bL > bR ? bL : bR;
            T esL = etaL + bL - Bs, esR = etaR + bR - Bs;
            if (esL < T(0)) esL = T(0);
            if (esR < T(0)) esR = T(0);
            const int k0 = 3 * ph;
            const T mL = etaL / (K.eps * c2L), mR = etaR / (K.eps * c2R);
            const T msL = esL / (K.eps * c2L), msR = esR / (K.eps * c2R);
            const T fL = mL > T(0) ? msL / mL : T(0), fR = mR > T(0) ? msR / mR : T(0);
            sL[k0] = msL;
            sL[k0 + 1] = uL[k0 + 1] * fL;
            sL[k0 + 2] = uL[k0 + 2] * fL;
            sR[k0] = msR;
            sR[k0 + 1] = uR[k0 + 1] * fR;
            sR[k0 + 2] = uR[k0 + 2] * fR;
            // the larger 1 / (eps c^2) of the two sides: each side's diffusion
            // covers its own flux m* v (no mass leaves a dry cell next to a wet
            // one on a different slope)
            dqm[ph] = (esR - esL) * ((c2L < c2R ? T(1) / c2L : T(1) / c2R) / K.eps);
            cL[k0] = mL;
            cL[k0 + 1] = uL[k0 + 1];
            cL[k0 + 2] = uL[k0 + 2];
            cR[k0] = mR;
            cR[k0 + 1] = uR[k0 + 1];
            cR[k0 + 2] = uR[k0 + 2];
        }
    }
    face_flux_sel(K, flags, sL, gL, sR, gR, d, H, T(1), T(1), dqm);
    T PL[NF], PLs[NF], PR[NF], PRs[NF];
    wb_pterm(K, cL, gL, d, PL);
    wb_pterm(K, sL, gL, d, PLs);
    wb_pterm(K, cR, gR, d, PR);
    wb_pterm(K, sR, gR, d, PRs);
#pragma unroll
    for (int k = 0; k < NF; k++) {
        cL[k] = PL[k] - PLs[k];
        cR[k] = PR[k] - PRs[k];
    }
}

// Savage-Hutter earth-pressure coefficients (Savage and Hutter 1989, in the
// two-dimensional form of Hutter et al. 1993) from c2 = cos^2 delta_int and
// t = tan delta_b: K_x = 2 (1 -/+ sqrt(1 - c2 (1 + t^2))) / c2 - 1 and
// K_y = (K_x + 1 -/+ sqrt((K_x - 1)^2 + 4 t^2)) / 2, the upper sign (active)
// where the flow extends along the direction, the lower (passive) where it is
// compressed.  ep_kmax is the largest value a cell can take (passive, then
// passive), the bound of the solid's pressure speed in the CFL step.
template <typename T>
M2P_FN T ep_kx(T c2, T t, bool active)
{
    const T disc = T(1) - c2 * (T(1) + t * t);
    const T r = sqrt(disc > T(0) ? disc : T(0));
    return T(2) * (active ? T(1) - r : T(1) + r) / c2 - T(1);
}
template <typename T>
M2P_FN T ep_ky(T kx, T t, bool active)
{
    const T r = sqrt((kx - T(1)) * (kx - T(1)) + T(4) * t * t);
    return T(0.5) * (active ? kx + T(1) - r : kx + T(1) + r);
}
template <typename T>
M2P_FN T ep_kmax(T c2, T t)
{
    return ep_ky(ep_kx(c2, t, false), t, false);
}

// Prescribed Mode-II face flux from the critical-depth inflow state
// (q, m_in, v_in, phi); sgn = +1 on W/S (inward +X/+Y), -1 on E/N.
template <typename T, bool H2 = false>
M2P_FN void inflow_flux(const Consts<T>& K, const Geo<T>& g, int d, int sgn, T q, T m_in,
                                            T v_in, T phi, T H[NF])
{
    T h = m_in / g.J, hs = phi * m_in / g.J;
    T Ns = g.c * (T(1) - K.al) * hs / T(2), pf = g.c * h / T(2);
    T Ax = d == 0 ? g.A11 : g.A21, Ay = d == 0 ? g.A12 : g.A22;
    T qs = phi * q, qf = (T(1) - phi) * q;
    H[0] = T(sgn) * qs;
    H[3] = T(sgn) * qf;
    H[1] = K.eps * g.J * h * Ax * Ns + (d == 0 ? qs * v_in : T(0));
    H[2] = K.eps * g.J * h * Ay * Ns + (d == 1 ? qs * v_in : T(0));
    H[4] = K.eps * g.J * h * Ax * pf + (d == 0 ? qf * v_in : T(0));
    H[5] = K.eps * g.J * h * Ay * pf + (d == 1 ? qf * v_in : T(0));
    if constexpr (carry_2h<T, H2>()) {
#pragma unroll
        for (int k = 0; k < NF; k++) H[k] = H[k] + H[k];
    }
}

// Viscous flux pieces at one face: J_b h and A_ij averaged over the two
// cells; normal derivative by the neighbour difference, tangential
// derivative as the mean of the two cells' central differences (cd*).
// x-face: FX = 2 Jh (A11 u_x + A21 u_y), FY = Jh (A12 u_x + A22 u_y + A11 w_x + A21 w_y).
template <typename T>
M2P_FN void visc_xface_c(T u0, T w0, T u1, T w1, T cdyu0, T cdyw0, T cdyu1, T cdyw1, T Jh0,
                                             T Jh1, const Geo<T>& ga, const Geo<T>& gb, T dxi, T& FX, T& FY)
{
    T dxu = (u1 - u0) / dxi, dxw = (w1 - w0) / dxi;
    T dyu = T(0.5) * (cdyu0 + cdyu1);
    T dyw = T(0.5) * (cdyw0 + cdyw1);
    T Jh = T(0.5) * (Jh0 + Jh1);
    T A11 = T(0.5) * (ga.A11 + gb.A11), A12 = T(0.5) * (ga.A12 + gb.A12);
    T A21 = T(0.5) * (ga.A21 + gb.A21), A22 = T(0.5) * (ga.A22 + gb.A22);
    FX = T(2) * Jh * (A11 * dxu + A21 * dyu);
    FY = Jh * (A12 * dxu + A22 * dyu + A11 * dxw + A21 * dyw);
}

// y-face: GX = Jh (A12 u_x + A22 u_y + A11 w_x + A21 w_y), GY = 2 Jh (A12 w_x + A22 w_y).
template <typename T>
M2P_FN void visc_yface_c(T u0, T w0, T u1, T w1, T cdxu0, T cdxw0, T cdxu1, T cdxw1, T Jh0,
                                             T Jh1, const Geo<T>& ga, const Geo<T>& gb, T deta, T& GX, T& GY)
{
    T dyu = (u1 - u0) / deta, dyw = (w1 - w0) / deta;
    T dxu = T(0.5) * (cdxu0 + cdxu1);
    T dxw = T(0.5) * (cdxw0 + cdxw1);
    T Jh = T(0.5) * (Jh0 + Jh1);
    T A11 = T(0.5) * (ga.A11 + gb.A11), A12 = T(0.5) * (ga.A12 + gb.A12);
    T A21 = T(0.5) * (ga.A21 + gb.A21), A22 = T(0.5) * (ga.A22 + gb.A22);
    GX = Jh * (A12 * dxu + A22 * dyu + A11 * dxw + A21 * dyw);
    GY = T(2) * Jh * (A12 * dxw + A22 * dyw);
}

// central difference of a neighbour pair over 2 h
template <typename T>
M2P_FN T cdiff(T up, T dn, T h)
{
    return (up - dn) / (T(2) * h);
}

// J_b h pbar^f with pbar^f = c h / 2.
template <typename T>
M2P_FN T fluid_G(T ms, T mf, const Geo<T>& g)
{
    if constexpr (Folded<T>::value) {
        // J_b c = 1: J_b h (c h / 2) = (c (m^s + m^f))^2 / 2
        const T hc = (ms + mf) * g.c;
        return T(0.5) * hc * hc;
    }
    T h = (ms + mf) / g.J;
    return g.J * h * (g.c * h / T(2));
}

// Source terms at a cell from the stage-input state, except the viscous term
// and the Coulomb friction (applied as a clamp after the update).
// dn: dn/dxi (3) then dn/deta (3).  dGx, dGy: central differences of fluid_G.
// Out: S[ph][a] accumulated in the order s_n, s_f, s_v, s_d (fluid only);
// kappa_s for the friction clamp; phif for the viscous prefactor.
// Centripetal term kappa = v_a (dn_a/dxi v_xi + dn_a/deta v_eta) of one phase
// from its velocities (v_xi, v_eta; v_Z by tangency) and the normal's
// derivatives dn (dn/dxi then dn/deta).
template <typename T>
M2P_FN T kappa_of(T v0, T v1, const Geo<T>& g, const T dn[6])
{
    const T v[3] = {v0, v1, g.bX * v0 + g.bY * v1};
    T k = T(0);
#pragma unroll
    for (int a = 0; a < 3; a++) k += v[a] * dn[a] * v0;
#pragma unroll
    for (int a = 0; a < 3; a++) k += v[a] * dn[3 + a] * v1;
    return k;
}

template <typename T>
struct Src {
    T sn[2][2], sf[2][2], sv[2][2], sd[2];
    T kappa_s, phif;
};

// wbs (the well-balanced option): per phase and direction, the balanced
// form -(fac / eps) (mean of the cell's two face values of eta) (difference
// of its two bed face values) / step that replaces the hydrostatic part of
// the basal-pressure source where the phase rests on the bed (fac = 1 - alpha
// for the solid, 1 for the fluid).
template <typename T>
M2P_FN void sources(const Consts<T>& K, int flags, const T u[NF], const Geo<T>& g,
                                        const T dn[6], T dGx, T dGy, Src<T>& S, const T* wbs = nullptr)
{
    if constexpr (Folded<T>::value) {
        _Pragma("clang fp contract(fast)")
        const T ms = u[0], mf = u[3];
        const T hs = ms * g.c, hf = mf * g.c;
        const T mt = ms + mf;
        T phis, phif;
        dsg2(ms, mf, mt, K.md, phis, phif);
        T v[2][3];
        dsg2(u[1], u[2], ms, K.md, v[0][0], v[0][1]);
        dsg2(u[4], u[5], mf, K.md, v[1][0], v[1][1]);
#pragma unroll
        for (int ph = 0; ph < 2; ph++) v[ph][2] = g.bX * v[ph][0] + g.bY * v[ph][1];
        T kap[2];
#pragma unroll
        for (int ph = 0; ph < 2; ph++) {
            const T ka = v[ph][0] * dn[0] + v[ph][1] * dn[3];
            const T kb = v[ph][0] * dn[1] + v[ph][1] * dn[4];
            const T kc = v[ph][0] * dn[2] + v[ph][1] * dn[5];
            kap[ph] = v[ph][0] * ka + v[ph][1] * kb + v[ph][2] * kc;
        }
        T pbs = hs * (g.c * K.oma - K.eps_chi * kap[0]);
        T pbf = hf * (g.c - K.eps_chi * kap[1]);
        if (pbs < T(0)) pbs = T(0);
        if (pbf < T(0)) pbf = T(0);
        // J_b p_b n (horizontal part) = -p_b (b_X, b_Y)
        S.sn[0][0] = -pbs * g.bX;
        S.sn[0][1] = -pbs * g.bY;
        S.sn[1][0] = -pbf * g.bX;
        S.sn[1][1] = -pbf * g.bY;
        if (wbs) {
            // hydrostatic part of -p_b b_n: -h c fac b_n
#pragma unroll
            for (int ph = 0; ph < 2; ph++) {
                const T fac = ph == 0 ? K.oma : T(1);
                const T hph = ph == 0 ? hs : hf;
                if (!((ph == 0 ? pbs : pbf) > T(0))) continue;
#pragma unroll
                for (int d = 0; d < 2; d++) {
                    const T hydro = -(hph * g.c * fac) * (d == 0 ? g.bX : g.bY);
                    S.sn[ph][d] = S.sn[ph][d] + (wbs[2 * ph + d] - hydro);
                }
            }
        }
        const T gx = g.A11 * dGx + g.A21 * dGy;
        const T gy = g.A12 * dGx + g.A22 * dGy;
        S.sf[0][0] = K.m_eps_al * phis * gx;
        S.sf[0][1] = K.m_eps_al * phis * gy;
        const T wf = (flags & 1) ? phif : phis;
        S.sf[1][0] = K.eps * wf * gx;
        S.sf[1][1] = K.eps * wf * gy;
        const T Kd = K.c_d * phis * phif * mt;  // J_b h = m^s + m^f
        const T dvx = v[1][0] - v[0][0], dvy = v[1][1] - v[0][1];
        S.sv[0][0] = K.al * Kd * dvx;
        S.sv[0][1] = K.al * Kd * dvy;
        S.sv[1][0] = -Kd * dvx;
        S.sv[1][1] = -Kd * dvy;
        const T fr = K.k_fr * phif * mt;
        S.sd[0] = -fr * v[1][0];
        S.sd[1] = -fr * v[1][1];
        S.kappa_s = kap[0];
        S.phif = phif;
        return;
    }
    T ms = u[0], mf = u[3];
    T hs = ms / g.J, hf = mf / g.J, h = hs + hf;
    T mt = ms + mf;
    T phis = dsg(ms, mt, K.md), phif = dsg(mf, mt, K.md);
    T v[2][2];
    v[0][0] = dsg(u[1], ms, K.md);
    v[0][1] = dsg(u[2], ms, K.md);
    v[1][0] = dsg(u[4], mf, K.md);
    v[1][1] = dsg(u[5], mf, K.md);
    T kap[2];
#pragma unroll
    for (int ph = 0; ph < 2; ph++) kap[ph] = kappa_of(v[ph][0], v[ph][1], g, dn);
    T pbs = hs * (g.c * (T(1) - K.al) - K.eps_chi * kap[0]);
    T pbf = hf * (g.c - K.eps_chi * kap[1]);
    if (pbs < T(0)) pbs = T(0);
    if (pbf < T(0)) pbf = T(0);
    S.sn[0][0] = g.J * pbs * g.nX;
    S.sn[0][1] = g.J * pbs * g.nY;
    S.sn[1][0] = g.J * pbf * g.nX;
    S.sn[1][1] = g.J * pbf * g.nY;
    if (wbs) {
        // hydrostatic part J_b h c fac n of J_b p_b n
#pragma unroll
        for (int ph = 0; ph < 2; ph++) {
            const T fac = ph == 0 ? T(1) - K.al : T(1);
            const T hph = ph == 0 ? hs : hf;
            if (!((ph == 0 ? pbs : pbf) > T(0))) continue;
#pragma unroll
            for (int d = 0; d < 2; d++) {
                const T hydro = g.J * hph * g.c * fac * (d == 0 ? g.nX : g.nY);
                S.sn[ph][d] += wbs[2 * ph + d] - hydro;
            }
        }
    }
    T gx = g.A11 * dGx + g.A21 * dGy;
    T gy = g.A12 * dGx + g.A22 * dGy;
    S.sf[0][0] = -K.eps * K.al * phis * gx;
    S.sf[0][1] = -K.eps * K.al * phis * gy;
    T wf = (flags & 1) ? phif : phis;
    S.sf[1][0] = K.eps * wf * gx;
    S.sf[1][1] = K.eps * wf * gy;
    T Kd = g.J * K.c_d * phis * phif * h;
    S.sv[0][0] = K.al * Kd * (v[1][0] - v[0][0]);
    S.sv[0][1] = K.al * Kd * (v[1][1] - v[0][1]);
    S.sv[1][0] = -Kd * (v[1][0] - v[0][0]);
    S.sv[1][1] = -Kd * (v[1][1] - v[0][1]);
    T fr = g.J * phif * h * K.theta_b * K.inv_n_r / K.eps;
    S.sd[0] = -fr * v[1][0];
    S.sd[1] = -fr * v[1][1];
    S.kappa_s = kap[0];
    S.phif = phif;
}

// Tentative forward-Euler update of one cell from its four face fluxes and
// its sources (summation order: x-difference, y-difference, then s_n, s_f,
// s_v, s_d^f, s_vis^f).
// cx, cy (the well-balanced option): per component, the cell's pressure
// corrections of its two faces in each direction, added to the flux differences.
template <typename T, bool H2 = false>
M2P_FN void tentative(const Consts<T>& K, const T u[NF], const T HXl[NF], const T HXr[NF],
                                          const T HYb[NF], const T HYt[NF], const Src<T>& S, T svx, T svy, T dt,
                                          T out[NF], const T* cx_wb = nullptr, const T* cy_wb = nullptr)
{
    if constexpr (carry_2h<T, H2>()) {
        _Pragma("clang fp contract(fast)")
        // fluxes carried as 2 H: u + dt s - (dt / 2 dxi) dF - (dt / 2 deta) dG
        const T cx = dt * K.half_rdxi, cy = dt * K.half_rdeta;
#pragma unroll
        for (int k = 0; k < NF; k++) {
            const T dFx = cx_wb ? (HXr[k] - HXl[k]) + cx_wb[k] : HXr[k] - HXl[k];
            const T dGy = cy_wb ? (HYt[k] - HYb[k]) + cy_wb[k] : HYt[k] - HYb[k];
            const int ph = k / 3, comp = k % 3;
            T o = u[k];
            if (comp > 0) {
                const int a = comp - 1;
                T sk = S.sn[ph][a] + S.sf[ph][a] + S.sv[ph][a];
                if (ph == 1) sk = sk + S.sd[a] + (a == 0 ? svx : svy);
                o = o + dt * sk;
            }
            o = o - cx * dFx;
            out[k] = o - cy * dGy;
        }
        return;
    }
    if constexpr (Folded<T>::value) {
        _Pragma("clang fp contract(fast)")
        // u + dt s - (dt / dxi) dF - (dt / deta) dG
        const T cx = dt * K.rdxi, cy = dt * K.rdeta;
#pragma unroll
        for (int k = 0; k < NF; k++) {
            const T dFx = cx_wb ? (HXr[k] - HXl[k]) + cx_wb[k] : HXr[k] - HXl[k];
            const T dGy = cy_wb ? (HYt[k] - HYb[k]) + cy_wb[k] : HYt[k] - HYb[k];
            const int ph = k / 3, comp = k % 3;
            T o = u[k];
            if (comp > 0) {
                const int a = comp - 1;
                T sk = S.sn[ph][a] + S.sf[ph][a] + S.sv[ph][a];
                if (ph == 1) sk = sk + S.sd[a] + (a == 0 ? svx : svy);
                o = o + dt * sk;
            }
            o = o - cx * dFx;
            out[k] = o - cy * dGy;
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < NF; k++) {
        T dFx = HXr[k] - HXl[k];
        T dGy = HYt[k] - HYb[k];
        if (cx_wb) dFx += cx_wb[k];
        if (cy_wb) dGy += cy_wb[k];
        T r = -dFx / K.dxi - dGy / K.deta;
        const int ph = k / 3, comp = k % 3;
        if (comp > 0) {
            const int a = comp - 1;
            r += S.sn[ph][a];
            r += S.sf[ph][a];
            r += S.sv[ph][a];
            if (ph == 1) {
                r += S.sd[a];
                r += a == 0 ? svx : svy;
            }
        }
        out[k] = u[k] + dt * r;
    }
}

// Coulomb stop-clamp of the solid momentum (basal pressure from the tentative
// solid thickness, centripetal term kappa_s from the stage input), then
// positivity: a phase with tentative thickness <= 0 loses its momentum.
// Returns the number of positivity clamps (tentative thickness < 0).
// SMOOTH = false leaves out the smooth-friction option (the fused stage
// kernels; contexts with the option run the reference kernel).
template <typename T, bool SMOOTH = true>
M2P_FN int clamp_cell(const Consts<T>& K, const Geo<T>& g, T kappa_s, T dt, T tmu, T out[NF])
{
    T F;
    if constexpr (Folded<T>::value) {
        _Pragma("clang fp contract(fast)")
        // J_b p_b = m^s (c (1 - alpha) - eps^chi kappa_s)
        T jpb = out[0] * (g.c * K.oma - K.eps_chi * kappa_s);
        if (jpb < T(0)) jpb = T(0);
        F = dt * jpb * tmu;
    } else {
        T hst = out[0] / g.J;
        T pbt = hst * (g.c * (T(1) - K.al) - K.eps_chi * kappa_s);
        if (pbt < T(0)) pbt = T(0);
        F = dt * (g.J * pbt) * tmu;
    }
    T pX = out[1], pY = out[2];
    T pZ = g.bX * pX + g.bY * pY;
    if (SMOOTH && K.smooth) {
        // smooth friction (gradient checks): p = p~ r / (r + F),
        // r = sqrt(|p~_3D|^2 + (m~^s v_eps)^2), a regularised Coulomb term
        // that never reverses the flow
        if (F > T(0)) {
            const T me = out[0] * K.veps;
            const T r = sqrt(pX * pX + pY * pY + pZ * pZ + me * me);
            out[1] = pX * (r / (r + F));
            out[2] = pY * (r / (r + F));
        }
    } else if constexpr (Folded<T>::value) {
        // |p_3| <= F  <=>  |p_3|^2 <= F^2 (F >= 0)
        const T p2 = pX * pX + pY * pY + pZ * pZ;
        if (p2 <= F * F) {
            out[1] = T(0);
            out[2] = T(0);
        } else {
            const T r = T(1) - F * rsq(p2);
            out[1] = pX * r;
            out[2] = pY * r;
        }
    } else {
        T p3 = sqrt(pX * pX + pY * pY + pZ * pZ);
        if (p3 <= F) {
            out[1] = T(0);
            out[2] = T(0);
        } else {
            out[1] = pX * (T(1) - F / p3);
            out[2] = pY * (T(1) - F / p3);
        }
    }
    int clamps = 0;
#pragma unroll
    for (int ph = 0; ph < 2; ph++)
        if (out[3 * ph] <= T(0)) {
            if (out[3 * ph] < T(0)) clamps++;
            out[3 * ph] = T(0);
            out[3 * ph + 1] = T(0);
            out[3 * ph + 2] = T(0);
        }
    return clamps;
}

template <typename T, bool H2 = false, bool SMOOTH = true>
M2P_FN int update_cell(const Consts<T>& K, const T u[NF], const Geo<T>& g, const T HXl[NF],
                                           const T HXr[NF], const T HYb[NF], const T HYt[NF], const Src<T>& S,
                                           T svx, T svy, T dt, T tmu, T out[NF], const T* cx_wb = nullptr,
                                           const T* cy_wb = nullptr)
{
    tentative<T, H2>(K, u, HXl, HXr, HYb, HYt, S, svx, svy, dt, out, cx_wb, cy_wb);
    return clamp_cell<T, SMOOTH>(K, g, S.kappa_s, dt, tmu, out);
}

// Ghost-cell index map (transmissive: copy the edge cell; wall: mirror with
// the normal momentum negated).
M2P_FN int map_index(int i, int n, int bc_lo, int bc_hi, int& flip)
{
    if (i < 0) {
        if (bc_lo == 1) {
            flip ^= 1;
            return -1 - i;
        }
        return 0;
    }
    if (i >= n) {
        if (bc_hi == 1) {
            flip ^= 1;
            return 2 * n - 1 - i;
        }
        return n - 1;
    }
    return i;
}

}  // namespace m2p
