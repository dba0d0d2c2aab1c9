// m2p_abi.hip -- the C ABI (include/m2p.h): argument validation, device
// memory, the padded DEM, scalar state on the device, and the step / run
// drivers that enqueue the per-precision kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <algorithm>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "m2p.h"
#include "m2p_host.h"
#include "m2p_launch.h"

using namespace m2p;

namespace m2p {

static thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return M2P_EHIP;
}

size_t round_up(size_t a, size_t m) { return (a + m - 1) / m * m; }

}  // namespace m2p

struct m2p_ctx {
    int dev = 0;
    hipStream_t stream = nullptr;
    int prec = M2P_FP64;
    size_t esz = 8;
    m2p_grid g{};
    m2p_params p{};
    KParams kp{};
    Bufs B{};
    bool own_state = true;
    bool has_state = false;
    bool dirty = true;
    bool poisoned = false;
    int variant = M2P_VARIANT_AUTO;
    int rows = 0;
    int slots = 0;  // resident wavefronts of the tiled stage kernel on the device
    Shape shape{};
    double* wpart = nullptr;
    size_t wcap = 0;  // per-wave partial slots the wpart buffer holds per stage
    size_t state_bytes = 0;
    void* b = nullptr;
    void* mu = nullptr;
    DevScalars* S = nullptr;
    double* bpart = nullptr;
    double* tables = nullptr;
    std::vector<double> tab_flux, tab_state;  // host copies of the two kinds of Mode-II hydrograph tables
    int state_toff[MAX_SEG] = {};             // offsets of the state tables within tab_state
    double* mass_part = nullptr;
    double* staging = nullptr;  // FP64 field staging [7][ny][nx]
    // step chunks captured in a HIP graph (m2p_set_graph), recaptured when
    // the kernel arguments they were captured with change
    int graph_chunk = 32;
    hipGraphExec_t gexec = nullptr;
    int gsteps = 0;
    KParams g_kp{};
    Bufs g_B{};
    Shape g_shape{};
    // output snapshots (m2p_run_outputs): two device slots of the six output
    // fields, two pinned host slots and a copy stream (default priority)
    double* snap_dev[2] = {nullptr, nullptr};
    double* snap_host[2] = {nullptr, nullptr};
    hipStream_t copy_stream = nullptr;
    hipEvent_t snap_ready[2] = {nullptr, nullptr}, snap_copied[2] = {nullptr, nullptr};
    double t_end = std::numeric_limits<double>::infinity();
    // per-kernel HIP-event timing (m2p_set_profiling)
    bool prof = false;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    double prof_ms[3] = {0, 0, 0};
    int64_t prof_n = 0;
    double* scratch = nullptr;  // device address of this device's scratch array (m2p_loss_noalloc)
};

// ------------------------------------------- scratch of the allocation-free loss
//
// m2p_loss_noalloc keeps the loss kernel's per-block partial sums in a fixed
// device array (16 KiB on every GPU the library runs on, held until the
// process ends) instead of context memory or a hipMalloc.  In host code the
// array's name is a host-side stand-in, never a device address: its address
// on a device comes from hipGetSymbolAddress, looked up once per device with
// that device current, and only that address reaches kernels.
constexpr int kScratchDoubles = 2048;
static_assert(kMassBlocks <= kScratchDoubles, "the loss kernel's partial sums must fit the scratch array");
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of the scratch array on device dev (the current device).
static int scratch_address(int dev, double** out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(M2P_EINVAL, "device index outside the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return M2P_OK;
}

// Sum of part[0 .. n) by one thread in index order: the same additions in the
// same order as the host sum of m2p_loss, so both give the same bits.
__global__ void __launch_bounds__(64) k_sum_in_order(const double* __restrict__ part, int n, double* __restrict__ out)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double acc = 0.0;
    for (int q = 0; q < n; q++) acc += part[q];
    *out = acc;
}

// One part of a step on the buffers B (the context's, or the same with other
// state pointers).
static hipError_t step_part(m2p_ctx* c, const Bufs& B, int part)
{
    // every launch shape's partial slots must fit the buffer (m2p_set_variant
    // grows it before a shape needs more)
    if ((size_t)c->shape.nw > c->wcap || (size_t)B.nw_ref > c->wcap) return hipErrorInvalidValue;
    if (c->prec == M2P_FP64) return Launch<double>::step_part(c->kp, B, c->shape, c->stream, part);
    return Launch<float>::step_part(c->kp, B, c->shape, c->stream, part);
}

static hipError_t step_part(m2p_ctx* c, int part) { return step_part(c, c->B, part); }

// One step: the rk stage kernels, then the finalize (parts 0 .. rk).  With
// profiling, an event around every part (rk + 2 events per step).
static hipError_t do_step(m2p_ctx* c)
{
    const int np = c->kp.rk + 1;
    if (!c->prof) {
        for (int part = 0; part < np; part++) {
            hipError_t e = step_part(c, part);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    while (c->ev.size() < c->ev_used + np + 1) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        c->ev.push_back(e);
    }
    hipEvent_t* e = &c->ev[c->ev_used];
    c->ev_used += np + 1;
    hipError_t r = hipEventRecord(e[0], c->stream);
    for (int part = 0; part < np && r == hipSuccess; part++) {
        r = step_part(c, part);
        if (r == hipSuccess) r = hipEventRecord(e[part + 1], c->stream);
    }
    return r;
}

static hipError_t do_init(m2p_ctx* c)
{
    if (c->prec == M2P_FP64) return Launch<double>::init(c->kp, c->B, c->stream);
    return Launch<float>::init(c->kp, c->B, c->stream);
}

namespace m2p {

// Launch shape: the reference variant uses 64 x 4 blocks; the tiled variant
// one wavefront per (strip of 60 output columns, R rows), R from the size and
// occupancy rules below unless fixed; slots = wavefronts of the tiled stage
// kernel the device holds at once (0: unknown).
Shape make_shape(const KParams& P, int variant, int rows, int slots)
{
    Shape s{};
    // the smooth-friction option, and earth pressure with the central-upwind
    // flux or with Mode-II state segments, and the well-balanced option with
    // state segments, run on the reference kernel
    const bool ep_ref =
        (P.flags & kFlagEarthPressure) && ((P.flags & kFlagCentralUpwind) || P.nsseg > 0);
    const bool wb_ref = (P.flags & kFlagWellBalanced) && P.nsseg > 0;
    s.variant = (variant == M2P_VARIANT_REFERENCE || (P.flags & kFlagSmoothFriction) || ep_ref || wb_ref) ? 1 : 2;
    s.global_addr = variant == M2P_VARIANT_TILED_GLOBAL;
    s.nbx = (P.nx + 63) / 64;
    s.nby = (P.ny + 3) / 4;
    s.nstrips = (P.nx + 59) / 60;
    int R = rows;
    if (R <= 0) {
        // A wavefront's march costs its R rows plus a prologue of about two
        // rows' work (the stencil window), so the redundant work falls like
        // 1/R while the latency of one wavefront grows like R; their sum is
        // least near R ~ sqrt(wave-rows).  The constant is the measured
        // optimum of FP32 runs from 100 x 100 to 4096 x 4096.
        const double wave_rows = (double)s.nstrips * P.ny;
        R = (int)std::lround(std::sqrt(wave_rows) / 22.0);
        R = R < 1 ? 1 : (R > 64 ? 64 : R);
        // The wavefronts run in rounds of `slots`.  When the last round would
        // be more than half full, the fewest rows per wavefront that leave it
        // out (at most 1.5 R) finish sooner: at 4096 x 4096 in FP32, 31 rows
        // (2.99 rounds) instead of 24 (3.84 rounds), 2 % per step.
        if (slots > 0) {
            const long nw = (long)s.nstrips * ((P.ny + R - 1) / R);
            const long full = nw / slots;
            if (full >= 1 && 2 * (nw - full * slots) > slots) {
                const long rb = full * slots / s.nstrips;  // row blocks that fit in the full rounds
                const long R2 = rb >= 1 ? (P.ny + rb - 1) / rb : 0;
                if (R2 > R && 2 * R2 <= 3 * R && R2 <= 64) R = (int)R2;
            }
        }
    }
    s.R = R;
    s.nrb = (P.ny + R - 1) / R;
    s.n_we = P.ny;  // one outflow slot per boundary face
    s.n_sn = P.nx;
    if (s.variant == 1) {
        s.nw = s.nbx * s.nby;
        s.blocks = s.nbx * s.nby;
    } else {
        s.blocks = (s.nstrips * s.nrb + 3) / 4;
        s.nw = s.blocks;  // one partial record per workgroup of four wavefronts
    }
    return s;
}

}  // namespace m2p

static void refresh_grid(m2p_ctx* c) { c->shape = make_shape(c->kp, c->variant, c->rows, c->slots); }

// Grow the per-wave partial buffer to the current launch shape (3 stage slots
// of 4 values per wave).  Contents start at zero; the finalize reads only the
// slots the last stage launches wrote.
static int ensure_wpart(m2p_ctx* c)
{
    const size_t need = std::max((size_t)c->shape.nw, (size_t)c->B.nw_ref);
    if (need <= c->wcap) return M2P_OK;
    double* w = nullptr;
    if (hipMalloc(&w, sizeof(double) * 3 * 4 * need) != hipSuccess)
        return fail(M2P_ENOMEM, "partials allocation failed");
    if (hipMemset(w, 0, sizeof(double) * 3 * 4 * need) != hipSuccess) {
        (void)hipFree(w);
        return fail(M2P_EHIP, "partials initialisation failed");
    }
    if (c->wpart) (void)hipFree(c->wpart);
    c->wpart = w;
    c->B.wpart = w;
    c->wcap = need;
    return M2P_OK;
}

static int ensure_ready(m2p_ctx* c)
{
    if (c->poisoned) return fail(M2P_ESTATE, "context poisoned by an earlier device error");
    if (!c->has_state) return fail(M2P_ESTATE, "no state: call m2p_set_state first");
    if (c->dirty) {
        double tend = c->t_end / c->kp.T;
        HIPCHK(hipMemcpyAsync(&c->S->t_end, &tend, sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIPCHK(do_init(c));
        c->dirty = false;
    }
    return M2P_OK;
}

static int check_status(m2p_ctx* c, const DevScalars& hs)
{
    if (hs.status & 1u) {
        c->poisoned = true;
        return fail(M2P_ENONFINITE, "non-finite value in the state or in dt");
    }
    if (hs.status & 2u) {
        c->poisoned = true;
        return fail(M2P_EDTFLOOR, "CFL time step below the floor");
    }
    return M2P_OK;
}

static int read_scalars(m2p_ctx* c, DevScalars* hs)
{
    HIPCHK(hipMemcpyAsync(hs, c->S, sizeof(DevScalars), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return M2P_OK;
}

namespace m2p {

// Dimensionless constants of a scenario (Sect. 2.2 scheme, Appendix A model).
KParams make_kparams(const m2p_grid* g, const m2p_params* p, bool has_mu)
{
    KParams K;
    std::memset(&K, 0, sizeof(K));
    K.nx = g->nx;
    K.ny = g->ny;
    K.pitch = (int)round_up((size_t)g->nx, 64);
    K.bpitch = (int)(BOFF + round_up((size_t)g->nx + BHALO, 64));
    for (int s = 0; s < 4; s++) K.bc[s] = p->bc[s];
    K.flags = p->flags;
    K.rk = (p->flags & M2P_F_RK3) ? 3 : 2;
    K.has_mu = has_mu ? 1 : 0;
    K.visc = p->inv_n_r != 0.0 ? 1 : 0;
    K.eps = p->H / p->L;
    K.alpha = p->rho_f / p->rho_s;
    K.one_m_alpha = 1.0 - K.alpha;
    K.dxi = g->dx / p->L;
    K.deta = g->dy / p->L;
    K.two_dxi = 2.0 * K.dxi;
    K.two_deta = 2.0 * K.deta;
    K.md = p->m_dry / p->H;
    K.eps_chi = std::pow(K.eps, p->chi);
    K.tan_d = std::tan(p->delta_b_deg * M_PI / 180.0);
    if (p->flags & M2P_F_EARTH_PRESSURE) {
        const double ci = std::cos(p->delta_int_deg * M_PI / 180.0);
        K.cos2_int = ci * ci;
    }
    K.c_d = p->c_d;
    K.inv_n_r = p->inv_n_r;
    K.theta_b = p->theta_b;
    K.T = std::sqrt(p->L / p->g);
    K.V = std::sqrt(p->g * p->L);
    K.H = p->H;
    K.L = p->L;
    K.dx = g->dx;
    K.dy = g->dy;
    K.cfl = p->cfl;
    K.a_floor = p->a_min / K.V;
    K.v_eps = (p->flags & M2P_F_SMOOTH_FRICTION) ? p->v_eps / K.V : 0.0;
    K.dt_floor = 1e-12 * std::min(K.dxi, K.deta) / std::sqrt(K.eps);
    return K;
}

// Padded DEM (b / L) with the two-cell ring continued by linear
// extrapolation: along Y for every column, then along X for every row.
std::vector<double> padded_dem(const KParams& K, const double* dem, double L)
{
    const int nx = K.nx, ny = K.ny, bp = K.bpitch;
    std::vector<double> bd((size_t)(ny + 2 * BHALO) * bp, 0.0);
    auto B = [&](int i, int j) -> double& { return bd[(size_t)(j + BHALO) * bp + BOFF + i]; };
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) B(i, j) = dem[(size_t)j * nx + i] / L;
    for (int i = 0; i < nx; i++) {
        double b0 = B(i, 0), b1 = B(i, 1), bn = B(i, ny - 1), bm = B(i, ny - 2);
        for (int k = 1; k <= BHALO; k++) {
            B(i, -k) = b0 + (double)(-k) * (b1 - b0);
            B(i, ny - 1 + k) = bn + (double)k * (bn - bm);
        }
    }
    for (int j = -BHALO; j < ny + BHALO; j++) {
        double b0 = B(0, j), b1 = B(1, j), bn = B(nx - 1, j), bm = B(nx - 2, j);
        for (int k = 1; k <= BHALO; k++) {
            B(-k, j) = b0 + (double)(-k) * (b1 - b0);
            B(nx - 1 + k, j) = bn + (double)k * (bn - bm);
        }
    }
    return bd;
}

// With the earth-pressure option every basal friction must stay at or below
// the internal friction (the coefficients are real only there).
int ep_friction_ok(const m2p_params* p, const double* tan_mu, size_t n)
{
    const double ti = std::tan(p->delta_int_deg * M_PI / 180.0);
    for (size_t k = 0; k < n; k++)
        if (!(tan_mu[k] <= ti)) return fail(M2P_EINVAL, "earth pressure needs tan(delta_b) <= tan(delta_int) everywhere");
    return M2P_OK;
}

int validate_scenario(const m2p_grid* g, const m2p_params* p, int32_t prec, const double* dem)
{
    if (!g || !p || !dem) return fail(M2P_EINVAL, "NULL argument");
    if (g->nx < 4 || g->ny < 4) return fail(M2P_EINVAL, "grid must be at least 4 x 4");
    if ((int64_t)g->nx * (int64_t)g->ny > (int64_t)1 << 31) return fail(M2P_EINVAL, "grid too large");
    if (!(g->dx > 0) || !(g->dy > 0) || !std::isfinite(g->dx) || !std::isfinite(g->dy))
        return fail(M2P_EINVAL, "dx, dy must be positive");
    if (prec != M2P_FP64 && prec != M2P_FP32) return fail(M2P_EINVAL, "precision must be M2P_FP64 or M2P_FP32");
    if (!(p->delta_b_deg >= 0.0 && p->delta_b_deg < 90.0)) return fail(M2P_EINVAL, "delta_b outside [0, 90)");
    if (!(p->cfl > 0.0 && p->cfl <= 1.0)) return fail(M2P_EINVAL, "cfl outside (0, 1]");
    if (!(p->rho_s > 0.0) || !(p->rho_f >= 0.0) || !(p->rho_f < p->rho_s))
        return fail(M2P_EINVAL, "densities must satisfy 0 <= rho_f < rho_s");
    if (!(p->L > 0.0) || !(p->H > 0.0) || !(p->g > 0.0)) return fail(M2P_EINVAL, "L, H, g must be positive");
    if (!(p->c_d >= 0.0) || !(p->inv_n_r >= 0.0) || !(p->theta_b >= 0.0) || !(p->m_dry > 0.0) ||
        !(p->a_min > 0.0) || !std::isfinite(p->chi))
        return fail(M2P_EINVAL, "c_d, 1/N_R, theta_b >= 0 and m_dry, a_min > 0 required");
    for (int s = 0; s < 4; s++)
        if (p->bc[s] != M2P_BC_TRANSMISSIVE && p->bc[s] != M2P_BC_WALL) return fail(M2P_EINVAL, "bad boundary mode");
    if (p->flags & ~(M2P_F_FLUID_PRESSURE_AS_PRINTED | M2P_F_RK3 | M2P_F_CENTRAL_UPWIND | M2P_F_EARTH_PRESSURE |
                     M2P_F_SMOOTH_FRICTION | M2P_F_WELL_BALANCED))
        return fail(M2P_EINVAL, "unknown flag");
    if ((p->flags & M2P_F_WELL_BALANCED) && (p->flags & M2P_F_EARTH_PRESSURE))
        return fail(M2P_EINVAL, "the well-balanced option is not combined with earth pressure");
    if ((p->flags & M2P_F_SMOOTH_FRICTION) && !(p->v_eps > 0.0 && std::isfinite(p->v_eps)))
        return fail(M2P_EINVAL, "smooth friction needs v_eps > 0");
    if ((p->flags & M2P_F_EARTH_PRESSURE) &&
        !(p->delta_int_deg >= 0.0 && p->delta_int_deg < 90.0 && p->delta_b_deg <= p->delta_int_deg))
        return fail(M2P_EINVAL, "earth pressure needs delta_b <= delta_int < 90 deg");
    size_t n = (size_t)g->nx * g->ny;
    for (size_t k = 0; k < n; k++)
        if (!std::isfinite(dem[k])) return fail(M2P_EINVAL, "non-finite DEM value");
    return M2P_OK;
}

}  // namespace m2p

extern "C" {

const char* m2p_version(void) { return "m2p 0.1 (gfx950)"; }

const char* m2p_strerror(int code)
{
    switch (code) {
        case M2P_OK: return "ok";
        case M2P_EINVAL: return "invalid argument";
        case M2P_ENOMEM: return "out of device memory";
        case M2P_EHIP: return "HIP runtime error";
        case M2P_ENONFINITE: return "non-finite value on the device";
        case M2P_ENEGDEPTH: return "negative thickness";
        case M2P_EDTFLOOR: return "time step below floor";
        case M2P_EMAXSTEPS: return "maximum number of steps reached";
        case M2P_ESTATE: return "invalid call order or poisoned context";
        case M2P_EIO: return "file input/output error";
        default: return "unknown status";
    }
}

const char* m2p_last_error(void) { return m2p::g_err.c_str(); }

int m2p_device_count(int* count)
{
    if (!count) return fail(M2P_EINVAL, "count is NULL");
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    *count = e == hipSuccess ? n : 0;
    return M2P_OK;
}

int m2p_buffer_bytes(const m2p_grid* g, int32_t prec, size_t* state_bytes)
{
    if (!g || !state_bytes) return fail(M2P_EINVAL, "NULL argument");
    if (g->nx < 4 || g->ny < 4) return fail(M2P_EINVAL, "grid must be at least 4 x 4");
    if (prec != M2P_FP64 && prec != M2P_FP32) return fail(M2P_EINVAL, "precision must be M2P_FP64 or M2P_FP32");
    size_t esz = prec == M2P_FP64 ? 8 : 4;
    *state_bytes = (size_t)NF * (size_t)g->ny * round_up((size_t)g->nx, 64) * esz;
    return M2P_OK;
}

int m2p_create(m2p_ctx** out, const m2p_grid* g, const m2p_params* p, int32_t prec, const double* dem,
               const double* tan_mu, void* hip_stream)
{
    if (!out) return fail(M2P_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_scenario(g, p, prec, dem);
    if (rc) return rc;
    const size_t n = (size_t)g->nx * g->ny;
    if (tan_mu)
        for (size_t k = 0; k < n; k++)
            if (!(tan_mu[k] >= 0.0) || !std::isfinite(tan_mu[k])) return fail(M2P_EINVAL, "bad tan_mu value");
    if (tan_mu && (p->flags & M2P_F_EARTH_PRESSURE) && (rc = ep_friction_ok(p, tan_mu, n))) return rc;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(M2P_EHIP, "no HIP device");
    m2p_ctx* c = new m2p_ctx();
    HIPCHK(hipGetDevice(&c->dev));
    c->stream = (hipStream_t)hip_stream;
    c->prec = prec;
    c->esz = prec == M2P_FP64 ? 8 : 4;
    c->g = *g;
    c->p = *p;
    c->kp = make_kparams(g, p, tan_mu != nullptr);
    c->slots = prec == M2P_FP64 ? Launch<double>::resident_waves(c->kp) : Launch<float>::resident_waves(c->kp);
    const KParams& K = c->kp;
    const int nx = g->nx, ny = g->ny;
    std::vector<double> bd = padded_dem(K, dem, p->L);
    auto cleanup = [&](int code) {
        m2p_destroy(c);
        return code;
    };
    size_t bbytes = bd.size() * c->esz;
    if (hipMalloc(&c->b, bbytes) != hipSuccess) return cleanup(fail(M2P_ENOMEM, "DEM allocation failed"));
    if (c->prec == M2P_FP64) {
        if (hipMemcpy(c->b, bd.data(), bbytes, hipMemcpyHostToDevice) != hipSuccess)
            return cleanup(fail(M2P_EHIP, "DEM copy failed"));
    } else {
        std::vector<float> bf(bd.begin(), bd.end());
        if (hipMemcpy(c->b, bf.data(), bbytes, hipMemcpyHostToDevice) != hipSuccess)
            return cleanup(fail(M2P_EHIP, "DEM copy failed"));
    }
    if (tan_mu) {
        size_t mb = (size_t)ny * K.pitch * c->esz;
        if (hipMalloc(&c->mu, mb) != hipSuccess) return cleanup(fail(M2P_ENOMEM, "friction field allocation failed"));
        std::vector<double> md((size_t)ny * K.pitch, 0.0);
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) md[(size_t)j * K.pitch + i] = tan_mu[(size_t)j * nx + i];
        hipError_t e;
        if (c->prec == M2P_FP64)
            e = hipMemcpy(c->mu, md.data(), mb, hipMemcpyHostToDevice);
        else {
            std::vector<float> mf(md.begin(), md.end());
            e = hipMemcpy(c->mu, mf.data(), mb, hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) return cleanup(fail(M2P_EHIP, "friction field copy failed"));
    }
    if (hipMalloc(&c->S, sizeof(DevScalars)) != hipSuccess) return cleanup(fail(M2P_ENOMEM, "scalar allocation failed"));
    DevScalars hs;
    std::memset(&hs, 0, sizeof(hs));
    hs.t_end = std::numeric_limits<double>::infinity();
    if (hipMemcpy(c->S, &hs, sizeof(hs), hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(M2P_EHIP, "scalar init failed"));
    refresh_grid(c);
    // partial buffers: outflow slots, one per boundary face; per-wave slots
    // for the reference blocks and the default tiled shape (m2p_set_variant
    // grows them for shorter tiles)
    {
        const int nmax = std::max(nx, ny) + 1;
        c->B.nmax = nmax;
        c->B.nw_ref = ((nx + 63) / 64) * ((ny + 3) / 4);
        if (hipMalloc(&c->bpart, sizeof(double) * (outflow_dt_index(nmax) + 2)) != hipSuccess)
            return cleanup(fail(M2P_ENOMEM, "partials allocation failed"));
        if (hipMemset(c->bpart, 0, sizeof(double) * (outflow_dt_index(nmax) + 2)) != hipSuccess)
            return cleanup(fail(M2P_EHIP, "partials initialisation failed"));
        if (ensure_wpart(c) != M2P_OK) return cleanup(M2P_ENOMEM);
    }
    if (hipMalloc(&c->mass_part, sizeof(double) * 2 * kMassBlocks) != hipSuccess)
        return cleanup(fail(M2P_ENOMEM, "partials allocation failed"));

    if (hipMalloc(&c->staging, sizeof(double) * 7 * n) != hipSuccess)
        return cleanup(fail(M2P_ENOMEM, "staging allocation failed"));
    if (hipMalloc(&c->tables, sizeof(double) * 8) != hipSuccess)
        return cleanup(fail(M2P_ENOMEM, "table allocation failed"));
    if ((p->flags & M2P_F_EARTH_PRESSURE) && hipMalloc(&c->B.kep, 2 * (size_t)ny * K.pitch * c->esz) != hipSuccess)
        return cleanup(fail(M2P_ENOMEM, "earth-pressure allocation failed"));
    m2p_buffer_bytes(g, prec, &c->state_bytes);
    c->B.b = c->b;
    c->B.mu = c->mu;
    c->B.S = c->S;
    c->B.bpart = c->bpart;
    c->B.wpart = c->wpart;
    c->B.tables = c->tables;
    c->B.mass_part = c->mass_part;
    // this device's scratch array (the context's device is current here)
    if ((rc = scratch_address(c->dev, &c->scratch)) != M2P_OK) return cleanup(rc);
    *out = c;
    return M2P_OK;
}

void m2p_destroy(m2p_ctx* c)
{
    if (!c) return;
    if (c->stream)
        (void)hipStreamSynchronize(c->stream);
    else
        (void)hipDeviceSynchronize();
    if (c->own_state) {
        if (c->B.U) (void)hipFree(c->B.U);
        if (c->B.Us) (void)hipFree(c->B.Us);
    }
    if (c->B.Us2) (void)hipFree(c->B.Us2);
    if (c->b) (void)hipFree(c->b);
    if (c->mu) (void)hipFree(c->mu);
    if (c->S) (void)hipFree(c->S);
    if (c->bpart) (void)hipFree(c->bpart);
    if (c->wpart) (void)hipFree(c->wpart);
    if (c->tables) (void)hipFree(c->tables);
    if (c->mass_part) (void)hipFree(c->mass_part);
    if (c->staging) (void)hipFree(c->staging);
    if (c->B.kep) (void)hipFree(c->B.kep);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    if (c->copy_stream) (void)hipStreamSynchronize(c->copy_stream);
    for (int q = 0; q < 2; q++) {
        if (c->snap_dev[q]) (void)hipFree(c->snap_dev[q]);
        if (c->snap_host[q]) (void)hipHostFree(c->snap_host[q]);
        if (c->snap_ready[q]) (void)hipEventDestroy(c->snap_ready[q]);
        if (c->snap_copied[q]) (void)hipEventDestroy(c->snap_copied[q]);
    }
    if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    delete c;
}

// The three-stage method's second stage state, always owned by the context.
static int ensure_stage_buffer(m2p_ctx* c)
{
    if (c->kp.rk != 3 || c->B.Us2) return M2P_OK;
    if (hipMalloc(&c->B.Us2, c->state_bytes) != hipSuccess) return fail(M2P_ENOMEM, "state allocation failed");
    HIPCHK(hipMemsetAsync(c->B.Us2, 0, c->state_bytes, c->stream));
    return M2P_OK;
}

int m2p_bind_buffers(m2p_ctx* c, void* a, void* b, size_t bytes)
{
    if (!c || !a || !b) return fail(M2P_EINVAL, "NULL argument");
    if (c->B.U) return fail(M2P_ESTATE, "buffers already set");
    if (bytes < c->state_bytes) return fail(M2P_EINVAL, "buffers too small");
    if (((uintptr_t)a & 255) || ((uintptr_t)b & 255)) return fail(M2P_EINVAL, "buffers must be 256-byte aligned");
    c->B.U = a;
    c->B.Us = b;
    c->own_state = false;
    HIPCHK(hipMemsetAsync(a, 0, c->state_bytes, c->stream));
    HIPCHK(hipMemsetAsync(b, 0, c->state_bytes, c->stream));
    return ensure_stage_buffer(c);
}

static int ensure_state_buffers(m2p_ctx* c)
{
    if (c->B.U) return M2P_OK;
    if (hipMalloc(&c->B.U, c->state_bytes) != hipSuccess) return fail(M2P_ENOMEM, "state allocation failed");
    if (hipMalloc(&c->B.Us, c->state_bytes) != hipSuccess) return fail(M2P_ENOMEM, "state allocation failed");
    c->own_state = true;
    HIPCHK(hipMemsetAsync(c->B.U, 0, c->state_bytes, c->stream));
    HIPCHK(hipMemsetAsync(c->B.Us, 0, c->state_bytes, c->stream));
    return ensure_stage_buffer(c);
}

int m2p_set_state(m2p_ctx* c, int32_t kind, const double* h, const double* phi, const double* vxs, const double* vys,
                  const double* vxf, const double* vyf)
{
    if (!c || !h || !phi) return fail(M2P_EINVAL, "NULL argument");
    if (c->poisoned) return fail(M2P_ESTATE, "context poisoned");
    if (kind != M2P_DEPTH_NORMAL && kind != M2P_DEPTH_VERTICAL) return fail(M2P_EINVAL, "bad depth kind");
    const size_t n = (size_t)c->g.nx * c->g.ny;
    for (size_t k = 0; k < n; k++) {
        if (!std::isfinite(h[k])) return fail(M2P_EINVAL, "thickness must be finite");
        if (h[k] < 0.0) return fail(M2P_ENEGDEPTH, "negative thickness");
        if (!(phi[k] >= 0.0 && phi[k] <= 1.0)) return fail(M2P_EINVAL, "solid fraction outside [0, 1]");
    }
    const double* v[4] = {vxs, vys, vxf, vyf};
    for (int q = 0; q < 4; q++)
        if (v[q])
            for (size_t k = 0; k < n; k++)
                if (!std::isfinite(v[q][k])) return fail(M2P_EINVAL, "non-finite velocity");
    int rc = ensure_state_buffers(c);
    if (rc) return rc;
    std::vector<double> f(6 * n, 0.0);
    std::memcpy(f.data(), h, n * sizeof(double));
    std::memcpy(f.data() + n, phi, n * sizeof(double));
    int has_v = 0;
    for (int q = 0; q < 4; q++)
        if (v[q]) {
            std::memcpy(f.data() + (2 + q) * n, v[q], n * sizeof(double));
            has_v = 1;
        }
    HIPCHK(hipMemcpyAsync(c->staging, f.data(), 6 * n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if (c->prec == M2P_FP64) {
        HIPCHK(Launch<double>::set_state(c->kp, c->B, c->staging, kind == M2P_DEPTH_VERTICAL, has_v, c->stream));
    } else {
        HIPCHK(Launch<float>::set_state(c->kp, c->B, c->staging, kind == M2P_DEPTH_VERTICAL, has_v, c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    c->has_state = true;
    c->dirty = true;
    return M2P_OK;
}

int m2p_set_state_raw(m2p_ctx* c, const double* U)
{
    if (!c || !U) return fail(M2P_EINVAL, "NULL argument");
    if (c->poisoned) return fail(M2P_ESTATE, "context poisoned");
    int rc = ensure_state_buffers(c);
    if (rc) return rc;
    const int nx = c->g.nx, ny = c->g.ny, pitch = c->kp.pitch;
    const size_t n = (size_t)nx * ny;
    for (size_t k = 0; k < NF * n; k++)
        if (!std::isfinite(U[k])) return fail(M2P_EINVAL, "non-finite state value");
    if (c->prec == M2P_FP64) {
        std::vector<double> h((size_t)NF * ny * pitch, 0.0);
        for (int k = 0; k < NF; k++)
            for (int j = 0; j < ny; j++)
                std::memcpy(&h[((size_t)k * ny + j) * pitch], &U[k * n + (size_t)j * nx], nx * sizeof(double));
        HIPCHK(hipMemcpy(c->B.U, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
    } else {
        std::vector<float> h((size_t)NF * ny * pitch, 0.0f);
        for (int k = 0; k < NF; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) h[((size_t)k * ny + j) * pitch + i] = (float)U[k * n + (size_t)j * nx + i];
        HIPCHK(hipMemcpy(c->B.U, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    c->has_state = true;
    c->dirty = true;
    return M2P_OK;
}

int m2p_get_state_raw(m2p_ctx* c, double* U)
{
    if (!c || !U) return fail(M2P_EINVAL, "NULL argument");
    if (!c->has_state) return fail(M2P_ESTATE, "no state");
    const int nx = c->g.nx, ny = c->g.ny, pitch = c->kp.pitch;
    const size_t n = (size_t)nx * ny;
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->prec == M2P_FP64) {
        std::vector<double> h((size_t)NF * ny * pitch);
        HIPCHK(hipMemcpy(h.data(), c->B.U, h.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int k = 0; k < NF; k++)
            for (int j = 0; j < ny; j++)
                std::memcpy(&U[k * n + (size_t)j * nx], &h[((size_t)k * ny + j) * pitch], nx * sizeof(double));
    } else {
        std::vector<float> h((size_t)NF * ny * pitch);
        HIPCHK(hipMemcpy(h.data(), c->B.U, h.size() * sizeof(float), hipMemcpyDeviceToHost));
        for (int k = 0; k < NF; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) U[k * n + (size_t)j * nx + i] = h[((size_t)k * ny + j) * pitch + i];
    }
    return M2P_OK;
}

int m2p_set_time(m2p_ctx* c, double t)
{
    if (!c || !std::isfinite(t)) return fail(M2P_EINVAL, "bad argument");
    double tn = t / c->kp.T;
    HIPCHK(hipMemcpyAsync(&c->S->t, &tn, sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->dirty = true;
    return M2P_OK;
}

// Device table of both kinds of hydrographs: discharge segments first, then
// state segments (their offsets are shifted past the discharge tables).
static int upload_tables(m2p_ctx* c)
{
    std::vector<double> tab(c->tab_flux);
    const int shift = (int)tab.size();
    tab.insert(tab.end(), c->tab_state.begin(), c->tab_state.end());
    KParams& K = c->kp;
    for (int s = 0; s < K.nsseg; s++) K.sseg[s].toff = shift + c->state_toff[s];
    K.ntab = (int)tab.size();
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->tables) (void)hipFree(c->tables);
    c->tables = nullptr;
    size_t nb = std::max<size_t>(tab.size(), 8) * sizeof(double);
    if (hipMalloc(&c->tables, nb) != hipSuccess) return fail(M2P_ENOMEM, "table allocation failed");
    if (!tab.empty()) HIPCHK(hipMemcpy(c->tables, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
    c->B.tables = c->tables;
    c->dirty = true;
    return M2P_OK;
}

static bool overlaps(const SegDesc* a, int na, int side, int i0, int n)
{
    for (int q = 0; q < na; q++)
        if (a[q].side == side && i0 < a[q].i0 + a[q].ncells && a[q].i0 < i0 + n) return true;
    return false;
}

int m2p_set_inflow(m2p_ctx* c, const m2p_inflow* seg, int32_t nseg)
{
    if (!c || (nseg > 0 && !seg)) return fail(M2P_EINVAL, "NULL argument");
    if (nseg > 0 && (c->kp.flags & M2P_F_EARTH_PRESSURE))
        return fail(M2P_EINVAL, "the earth-pressure option runs Mode-I releases only");
    if (nseg > 0 && (c->kp.flags & M2P_F_WELL_BALANCED))
        return fail(M2P_EINVAL, "the well-balanced option takes Mode-II inflow as state segments only");
    if (nseg < 0 || nseg > MAX_SEG) return fail(M2P_EINVAL, "0..8 inflow segments supported");
    std::vector<double> tab;
    SegDesc sd[MAX_SEG];
    for (int s = 0; s < nseg; s++) {
        const m2p_inflow& q = seg[s];
        int len = q.side < 2 ? c->g.ny : c->g.nx;
        if (q.side < 0 || q.side > 3 || q.ncells < 1 || q.i0 < 0 || q.i0 + q.ncells > len || q.nt < 1 || !q.t ||
            !q.Q || !q.phi_s)
            return fail(M2P_EINVAL, "bad inflow segment");
        if (overlaps(sd, s, q.side, q.i0, q.ncells) || overlaps(c->kp.sseg, c->kp.nsseg, q.side, q.i0, q.ncells))
            return fail(M2P_EINVAL, "inflow segments overlap");
        for (int k = 0; k < q.nt; k++) {
            if (!std::isfinite(q.t[k]) || !(q.Q[k] >= 0.0) || !(q.phi_s[k] >= 0.0 && q.phi_s[k] <= 1.0))
                return fail(M2P_EINVAL, "bad hydrograph sample");
            if (k > 0 && !(q.t[k] > q.t[k - 1])) return fail(M2P_EINVAL, "hydrograph times must increase");
        }
        sd[s].side = q.side;
        sd[s].i0 = q.i0;
        sd[s].ncells = q.ncells;
        sd[s].nt = q.nt;
        sd[s].toff = (int)tab.size();
        tab.insert(tab.end(), q.t, q.t + q.nt);
        tab.insert(tab.end(), q.Q, q.Q + q.nt);
        tab.insert(tab.end(), q.phi_s, q.phi_s + q.nt);
    }
    KParams& K = c->kp;
    for (int s = 0; s < nseg; s++) K.seg[s] = sd[s];
    K.nseg = nseg;
    c->tab_flux = tab;
    return upload_tables(c);
}

int m2p_set_inflow_states(m2p_ctx* c, const m2p_inflow_state* seg, int32_t nseg)
{
    if (!c || (nseg > 0 && !seg)) return fail(M2P_EINVAL, "NULL argument");
    if (nseg > 0 && (c->kp.flags & M2P_F_EARTH_PRESSURE))
        return fail(M2P_EINVAL, "the earth-pressure option runs Mode-I releases only");
    if (nseg < 0 || nseg > MAX_SEG) return fail(M2P_EINVAL, "0..8 inflow state segments supported");
    std::vector<double> tab;
    SegDesc sd[MAX_SEG];
    for (int s = 0; s < nseg; s++) {
        const m2p_inflow_state& q = seg[s];
        int len = q.side < 2 ? c->g.ny : c->g.nx;
        if (q.side < 0 || q.side > 3 || q.ncells < 1 || q.i0 < 0 || q.i0 + q.ncells > len || q.nt < 1 || !q.t ||
            !q.h || !q.phi_s || !q.v)
            return fail(M2P_EINVAL, "bad inflow state segment");
        if (overlaps(sd, s, q.side, q.i0, q.ncells) || overlaps(c->kp.seg, c->kp.nseg, q.side, q.i0, q.ncells))
            return fail(M2P_EINVAL, "inflow segments overlap");
        for (int k = 0; k < q.nt; k++) {
            if (!std::isfinite(q.t[k]) || !(q.h[k] >= 0.0) || !std::isfinite(q.h[k]) ||
                !(q.phi_s[k] >= 0.0 && q.phi_s[k] <= 1.0) || !std::isfinite(q.v[k]))
                return fail(M2P_EINVAL, "bad hydrograph sample");
            if (k > 0 && !(q.t[k] > q.t[k - 1])) return fail(M2P_EINVAL, "hydrograph times must increase");
        }
        sd[s].side = q.side;
        sd[s].i0 = q.i0;
        sd[s].ncells = q.ncells;
        sd[s].nt = q.nt;
        sd[s].toff = (int)tab.size();
        tab.insert(tab.end(), q.t, q.t + q.nt);
        tab.insert(tab.end(), q.h, q.h + q.nt);
        tab.insert(tab.end(), q.phi_s, q.phi_s + q.nt);
        tab.insert(tab.end(), q.v, q.v + q.nt);
    }
    KParams& K = c->kp;
    for (int s = 0; s < nseg; s++) {
        K.sseg[s] = sd[s];
        c->state_toff[s] = sd[s].toff;
    }
    K.nsseg = nseg;
    c->tab_state = tab;
    // the kernel variant depends on whether state segments exist (options
    // that run them on the reference kernel)
    refresh_grid(c);
    if (int rc = ensure_wpart(c)) return rc;
    return upload_tables(c);
}

int m2p_set_variant(m2p_ctx* c, int32_t variant, int32_t rows)
{
    if (!c) return fail(M2P_EINVAL, "NULL context");
    if (variant < M2P_VARIANT_AUTO || variant > M2P_VARIANT_TILED_GLOBAL) return fail(M2P_EINVAL, "unknown variant");
    if (rows != 0 && (rows < 1 || rows > 4096)) return fail(M2P_EINVAL, "tile rows must be 0 or in [1, 4096]");
    HIPCHK(hipStreamSynchronize(c->stream));
    const int old_variant = c->variant, old_rows = c->rows;
    c->variant = variant;
    c->rows = rows;
    refresh_grid(c);
    const int rc = ensure_wpart(c);
    if (rc != M2P_OK) {
        c->variant = old_variant;
        c->rows = old_rows;
        refresh_grid(c);
    }
    return rc;
}

int m2p_autotune(m2p_ctx* c, int32_t trial_steps, int32_t* rows_out, double* ms_out)
{
    if (!c || trial_steps < 1 || trial_steps > 10000) return fail(M2P_EINVAL, "bad argument");
    int rc = ensure_ready(c);
    if (rc) return rc;
    const Shape auto_shape = make_shape(c->kp, M2P_VARIANT_TILED, 0, c->slots);
    if (make_shape(c->kp, c->variant, c->rows, c->slots).variant != 2)
        return fail(M2P_EINVAL, "the reference kernel has no tile");
    // candidates around the size rule's height
    const int r0 = auto_shape.R;
    std::vector<int> cand;
    for (double f : {0.5, 0.67, 0.8, 1.0, 1.2, 1.33, 1.5, 1.75}) {
        const int r = std::max(1, std::min(64, (int)std::lround(r0 * f)));
        if (std::find(cand.begin(), cand.end(), r) == cand.end()) cand.push_back(r);
    }
    // the trials run on the context's own state: keep the state, the device
    // scalars and the outflow integrals, and put them back after each trial
    const size_t bbytes = sizeof(double) * 4 * 2 * (size_t)c->B.nmax;
    void *ub = nullptr, *sb = nullptr, *bb = nullptr;
    if (hipMalloc(&ub, c->state_bytes) != hipSuccess || hipMalloc(&sb, sizeof(DevScalars)) != hipSuccess ||
        hipMalloc(&bb, bbytes) != hipSuccess) {
        if (ub) (void)hipFree(ub);
        if (sb) (void)hipFree(sb);
        return fail(M2P_ENOMEM, "autotune backup allocation failed");
    }
    struct Free {
        void *a, *b, *c;
        ~Free()
        {
            (void)hipFree(a);
            (void)hipFree(b);
            (void)hipFree(c);
        }
    } free_bufs{ub, sb, bb};
    HIPCHK(hipMemcpyAsync(ub, c->B.U, c->state_bytes, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(sb, c->S, sizeof(DevScalars), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(bb, c->bpart, bbytes, hipMemcpyDeviceToDevice, c->stream));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const int old_variant = c->variant, old_rows = c->rows;
    const bool old_prof = c->prof;
    c->prof = false;
    double best = 1e300;
    int bestR = r0;
    for (int r : cand) {
        c->variant = M2P_VARIANT_TILED;
        c->rows = r;
        refresh_grid(c);
        if ((rc = ensure_wpart(c))) break;
        hipError_t e = do_step(c);  // warm
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        for (int k = 0; k < trial_steps && e == hipSuccess; k++) e = do_step(c);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess) e = hipMemcpyAsync(c->B.U, ub, c->state_bytes, hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(c->S, sb, sizeof(DevScalars), hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(c->bpart, bb, bbytes, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) {
            rc = hip_fail(e, "autotune trial");
            break;
        }
        if (ms < best) {
            best = ms;
            bestR = r;
        }
    }
    (void)hipStreamSynchronize(c->stream);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->prof = old_prof;
    if (rc) {
        c->variant = old_variant;
        c->rows = old_rows;
        refresh_grid(c);
        return rc;
    }
    c->variant = old_variant;
    c->rows = bestR;
    refresh_grid(c);
    if ((rc = ensure_wpart(c))) return rc;
    if (rows_out) *rows_out = bestR;
    if (ms_out) *ms_out = best / trial_steps;
    return M2P_OK;
}

int m2p_step(m2p_ctx* c, double* dt_out)
{
    if (!c) return fail(M2P_EINVAL, "NULL context");
    int rc = ensure_ready(c);
    if (rc) return rc;
    if (!dt_out) {
        HIPCHK(do_step(c));
        return M2P_OK;
    }
    DevScalars hs;
    rc = read_scalars(c, &hs);
    if (rc) return rc;
    const double dt = hs.dt;
    HIPCHK(do_step(c));
    rc = read_scalars(c, &hs);
    if (rc) return rc;
    rc = check_status(c, hs);
    if (rc) return rc;
    *dt_out = dt * c->kp.T;
    return M2P_OK;
}

// A graph of graph_chunk steps captured on the context's stream with the
// current kernel arguments (constants, buffers, launch shape).  Graphs need
// a stream of their own (not the null stream) and are not used while
// per-kernel profiling is on.
static bool graph_usable(const m2p_ctx* c) { return c->stream && !c->prof && c->graph_chunk > 0; }

static int ensure_graph(m2p_ctx* c)
{
    if (c->gexec && c->gsteps == c->graph_chunk && !std::memcmp(&c->g_kp, &c->kp, sizeof(KParams)) &&
        !std::memcmp(&c->g_B, &c->B, sizeof(Bufs)) && !std::memcmp(&c->g_shape, &c->shape, sizeof(Shape)))
        return M2P_OK;
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    hipGraph_t graph;
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < c->graph_chunk; k++) {
        const hipError_t e = do_step(c);
        if (e != hipSuccess) {
            (void)hipStreamEndCapture(c->stream, &graph);
            return hip_fail(e, "kernel launch during graph capture");
        }
    }
    HIPCHK(hipStreamEndCapture(c->stream, &graph));
    const hipError_t e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHK(e);
    c->gsteps = c->graph_chunk;
    std::memcpy(&c->g_kp, &c->kp, sizeof(KParams));
    std::memcpy(&c->g_B, &c->B, sizeof(Bufs));
    std::memcpy(&c->g_shape, &c->shape, sizeof(Shape));
    return M2P_OK;
}

// n steps: whole graph chunks, then single steps.
static int issue_steps(m2p_ctx* c, int64_t n)
{
    int64_t done = 0;
    if (graph_usable(c) && n >= c->graph_chunk) {
        const int rc = ensure_graph(c);
        if (rc) return rc;
        for (; done + c->gsteps <= n; done += c->gsteps) HIPCHK(hipGraphLaunch(c->gexec, c->stream));
    }
    for (; done < n; done++) HIPCHK(do_step(c));
    return M2P_OK;
}

int m2p_run(m2p_ctx* c, int64_t nsteps)
{
    if (!c || nsteps < 0) return fail(M2P_EINVAL, "bad argument");
    int rc = ensure_ready(c);
    if (rc) return rc;
    return issue_steps(c, nsteps);
}

int m2p_set_graph(m2p_ctx* c, int32_t chunk)
{
    if (!c || chunk < 0 || chunk > 4096) return fail(M2P_EINVAL, "graph chunk must be in [0, 4096]");
    HIPCHK(hipStreamSynchronize(c->stream));
    c->graph_chunk = chunk;
    return M2P_OK;
}

// Step until the model time reaches t_end (the last step shortened to land on
// it) or max_steps steps were issued; chunks of steps between host checks.
static int advance_to(m2p_ctx* c, double t_end, int64_t max_steps, int64_t* steps_done)
{
    *steps_done = 0;
    c->t_end = t_end;
    c->dirty = true;
    int rc = ensure_ready(c);
    if (rc) return rc;
    DevScalars hs;
    rc = read_scalars(c, &hs);
    if (rc) return rc;
    const long long s0 = hs.steps;
    const double tn_end = t_end / c->kp.T;
    int64_t issued = 0, chunk = 8;
    rc = M2P_OK;
    while (hs.t < tn_end) {
        if (issued >= max_steps) {
            rc = fail(M2P_EMAXSTEPS, "max_steps reached before t_end");
            break;
        }
        int64_t k = std::min<int64_t>(chunk, max_steps - issued);
        if ((rc = issue_steps(c, k))) break;
        issued += k;
        chunk = std::min<int64_t>(chunk * 2, 1024);
        rc = read_scalars(c, &hs);
        if (rc) break;
        rc = check_status(c, hs);
        if (rc) break;
        if (hs.dt == 0.0 && hs.t < tn_end) {
            rc = fail(M2P_EDTFLOOR, "zero time step before t_end");
            c->poisoned = true;
            break;
        }
    }
    *steps_done = hs.steps - s0;
    c->t_end = std::numeric_limits<double>::infinity();
    c->dirty = true;
    return rc;
}

int m2p_run_to(m2p_ctx* c, double t_end, int64_t max_steps, int64_t* steps_done)
{
    if (!c || !std::isfinite(t_end) || max_steps < 0) return fail(M2P_EINVAL, "bad argument");
    int64_t done = 0;
    const int rc = advance_to(c, t_end, max_steps, &done);
    if (steps_done) *steps_done = done;
    return rc;
}

static int ensure_snapshots(m2p_ctx* c)
{
    if (c->copy_stream) return M2P_OK;
    const size_t bytes = sizeof(double) * 6 * (size_t)c->g.nx * c->g.ny;
    for (int q = 0; q < 2; q++) {
        if (hipMalloc(&c->snap_dev[q], bytes) != hipSuccess) return fail(M2P_ENOMEM, "snapshot allocation failed");
        if (hipHostMalloc(&c->snap_host[q], bytes, hipHostMallocDefault) != hipSuccess)
            return fail(M2P_ENOMEM, "pinned snapshot allocation failed");
        HIPCHK(hipEventCreateWithFlags(&c->snap_ready[q], hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->snap_copied[q], hipEventDisableTiming));
    }
    HIPCHK(hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking));
    return M2P_OK;
}

int m2p_run_outputs(m2p_ctx* c, const double* t_out, int64_t n_out, int64_t max_steps, double* fields,
                    int64_t* steps_done)
{
    if (steps_done) *steps_done = 0;
    if (!c || !t_out || !fields || n_out < 1 || max_steps < 0) return fail(M2P_EINVAL, "bad argument");
    for (int64_t k = 0; k < n_out; k++)
        if (!std::isfinite(t_out[k]) || (k > 0 && !(t_out[k] > t_out[k - 1])))
            return fail(M2P_EINVAL, "output times must be finite and increasing");
    if (!c->has_state) return fail(M2P_ESTATE, "no state: call m2p_set_state first");
    int rc = ensure_snapshots(c);
    if (rc) return rc;
    const size_t slot = 6 * (size_t)c->g.nx * c->g.ny;
    int64_t pending[2] = {-1, -1}, total = 0;
    // host copy of the snapshot in slot q once its device-to-host copy is done
    auto drain = [&](int q) -> int {
        if (pending[q] < 0) return M2P_OK;
        HIPCHK(hipEventSynchronize(c->snap_copied[q]));
        std::memcpy(fields + (size_t)pending[q] * slot, c->snap_host[q], slot * sizeof(double));
        pending[q] = -1;
        return M2P_OK;
    };
    for (int64_t k = 0; k < n_out && rc == M2P_OK; k++) {
        int64_t done = 0;
        rc = advance_to(c, t_out[k], max_steps - total, &done);
        total += done;
        if (rc) break;
        const int q = (int)(k & 1);
        if ((rc = drain(q))) break;  // slot q held output k - 2
        if (c->prec == M2P_FP64) {
            HIPCHK(Launch<double>::get_fields(c->kp, c->B, c->snap_dev[q], c->stream));
        } else {
            HIPCHK(Launch<float>::get_fields(c->kp, c->B, c->snap_dev[q], c->stream));
        }
        HIPCHK(hipEventRecord(c->snap_ready[q], c->stream));
        HIPCHK(hipStreamWaitEvent(c->copy_stream, c->snap_ready[q], 0));
        HIPCHK(hipMemcpyAsync(c->snap_host[q], c->snap_dev[q], slot * sizeof(double), hipMemcpyDeviceToHost,
                              c->copy_stream));
        HIPCHK(hipEventRecord(c->snap_copied[q], c->copy_stream));
        pending[q] = k;
    }
    for (int64_t k = n_out - 2; k < n_out; k++) {
        if (k < 0) continue;
        const int r2 = drain((int)(k & 1));
        if (r2 && rc == M2P_OK) rc = r2;
    }
    if (steps_done) *steps_done = total;
    return rc;
}

int m2p_get_fields(m2p_ctx* c, double* h, double* phi, double* vxs, double* vys, double* vxf, double* vyf)
{
    if (!c) return fail(M2P_EINVAL, "NULL context");
    if (!c->has_state) return fail(M2P_ESTATE, "no state");
    const size_t n = (size_t)c->g.nx * c->g.ny;
    if (c->prec == M2P_FP64) {
        HIPCHK(Launch<double>::get_fields(c->kp, c->B, c->staging, c->stream));
    } else {
        HIPCHK(Launch<float>::get_fields(c->kp, c->B, c->staging, c->stream));
    }
    std::vector<double> f(6 * n);
    HIPCHK(hipMemcpyAsync(f.data(), c->staging, 6 * n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    double* o[6] = {h, phi, vxs, vys, vxf, vyf};
    for (int q = 0; q < 6; q++)
        if (o[q]) std::memcpy(o[q], f.data() + q * n, n * sizeof(double));
    return M2P_OK;
}

}  // extern "C"

namespace m2p {

// Outflow volumes (m^3) of both phases from the per-face running integrals
// ([4 sides][nmax][2]), summed on the host in a fixed order: side by side,
// face by face.
int outflow_volumes(const double* bpart_dev, int nmax, int nx, int ny, const KParams& K, hipStream_t st,
                    double* out_s, double* out_f)
{
    std::vector<double> acc((size_t)4 * nmax * 2);
    HIPCHK(hipMemcpyAsync(acc.data(), bpart_dev, acc.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double o[2] = {0.0, 0.0};
    for (int side = 0; side < 4; side++) {
        const int n = side < 2 ? ny : nx;
        for (int k = 0; k < n; k++)
            for (int ph = 0; ph < 2; ph++) o[ph] += acc[((size_t)side * nmax + k) * 2 + ph];
    }
    const double vs = K.H * K.L * K.L;  // dimensionless volume -> m^3
    *out_s = o[0] * vs;
    *out_f = o[1] * vs;
    return M2P_OK;
}

}  // namespace m2p

extern "C" {

int m2p_get_diag(m2p_ctx* c, m2p_diag* d)
{
    if (!c || !d) return fail(M2P_EINVAL, "NULL argument");
    std::memset(d, 0, sizeof(*d));
    DevScalars hs;
    int rc = read_scalars(c, &hs);
    if (rc) return rc;
    if (c->has_state) {
        if (c->prec == M2P_FP64) {
            HIPCHK(Launch<double>::mass(c->kp, c->B, c->stream));
        } else {
            HIPCHK(Launch<float>::mass(c->kp, c->B, c->stream));
        }
        std::vector<double> part(2 * kMassBlocks);
        HIPCHK(hipMemcpyAsync(part.data(), c->mass_part, part.size() * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        double ms = 0.0, mf = 0.0;
        for (int q = 0; q < kMassBlocks; q++) {
            ms += part[2 * q];
            mf += part[2 * q + 1];
        }
        const KParams& K = c->kp;
        double scale = K.H * K.L * K.L * K.dxi * K.deta;
        d->mass_s = ms * scale;
        d->mass_f = mf * scale;
    }
    d->t = hs.t * c->kp.T;
    d->dt_last = hs.dt_last * c->kp.T;
    d->dt_next = hs.dt * c->kp.T;
    d->in_s = hs.in_s;
    d->in_f = hs.in_f;
    rc = outflow_volumes(c->bpart, c->B.nmax, c->g.nx, c->g.ny, c->kp, c->stream, &d->out_s, &d->out_f);
    if (rc) return rc;
    d->steps = hs.steps;
    d->clamp_count = (int64_t)hs.clamps;
    d->status = (int32_t)hs.status;
    return M2P_OK;
}

int m2p_synchronize(m2p_ctx* c)
{
    if (!c) return fail(M2P_EINVAL, "NULL context");
    HIPCHK(hipStreamSynchronize(c->stream));
    return M2P_OK;
}

int m2p_set_profiling(m2p_ctx* c, int32_t on)
{
    if (!c) return fail(M2P_EINVAL, "NULL context");
    c->prof = on != 0;
    return M2P_OK;
}

int m2p_kernel_times(m2p_ctx* c, double* ms, int64_t* nsteps)
{
    if (!c || !ms || !nsteps) return fail(M2P_EINVAL, "NULL argument");
    HIPCHK(hipStreamSynchronize(c->stream));
    const int np = c->kp.rk + 1;
    for (size_t g = 0; g + np + 1 <= c->ev_used; g += np + 1) {
        for (int part = 0; part < np; part++) {
            float t = 0.0f;
            HIPCHK(hipEventElapsedTime(&t, c->ev[g + part], c->ev[g + part + 1]));
            // first stage, the other stages, finalize
            c->prof_ms[part == 0 ? 0 : (part == np - 1 ? 2 : 1)] += t;
        }
        c->prof_n++;
    }
    c->ev_used = 0;
    for (int part = 0; part < 3; part++) ms[part] = c->prof_ms[part];
    *nsteps = c->prof_n;
    c->prof_ms[0] = c->prof_ms[1] = c->prof_ms[2] = 0.0;
    c->prof_n = 0;
    return M2P_OK;
}

int m2p_state_device_ptr(m2p_ctx* c, void** ptr, int64_t* pitch)
{
    if (!c || !ptr || !pitch) return fail(M2P_EINVAL, "NULL argument");
    *ptr = c->B.U;
    *pitch = c->kp.pitch;
    return M2P_OK;
}

}  // extern "C"

// ------------------------------------------------------------ adjoint support

namespace {

struct DevBuf {
    void* p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    int alloc(size_t bytes)
    {
        if (hipMalloc(&p, bytes) != hipSuccess) return m2p::fail(M2P_ENOMEM, "device allocation failed");
        if (hipMemset(p, 0, bytes) != hipSuccess) return m2p::fail(M2P_EHIP, "device memset failed");
        return M2P_OK;
    }
};

// host [k][ny][nx] FP64 <-> device [k][ny][pitch] in the context precision
int upload(m2p_ctx* c, const double* h, void* d, int nfields)
{
    const int nx = c->g.nx, ny = c->g.ny, pitch = c->kp.pitch;
    const size_t n = (size_t)nx * ny;
    if (c->prec == M2P_FP64) {
        std::vector<double> v((size_t)nfields * ny * pitch, 0.0);
        for (int k = 0; k < nfields; k++)
            for (int j = 0; j < ny; j++)
                std::memcpy(&v[((size_t)k * ny + j) * pitch], &h[k * n + (size_t)j * nx], nx * sizeof(double));
        HIPCHK(hipMemcpy(d, v.data(), v.size() * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<float> v((size_t)nfields * ny * pitch, 0.0f);
        for (int k = 0; k < nfields; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) v[((size_t)k * ny + j) * pitch + i] = (float)h[k * n + (size_t)j * nx + i];
        HIPCHK(hipMemcpy(d, v.data(), v.size() * 4, hipMemcpyHostToDevice));
    }
    return M2P_OK;
}

int download(m2p_ctx* c, const void* d, double* h, int nfields)
{
    const int nx = c->g.nx, ny = c->g.ny, pitch = c->kp.pitch;
    const size_t n = (size_t)nx * ny, tot = (size_t)nfields * ny * pitch;
    HIPCHK(hipStreamSynchronize(c->stream));
    std::vector<double> v(tot);
    if (c->prec == M2P_FP64) {
        HIPCHK(hipMemcpy(v.data(), d, tot * 8, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> f(tot);
        HIPCHK(hipMemcpy(f.data(), d, tot * 4, hipMemcpyDeviceToHost));
        std::copy(f.begin(), f.end(), v.begin());
    }
    for (int k = 0; k < nfields; k++)
        for (int j = 0; j < ny; j++) std::memcpy(&h[k * n + (size_t)j * nx], &v[((size_t)k * ny + j) * pitch], nx * 8);
    return M2P_OK;
}

hipError_t L_jvp(m2p_ctx* c, const void* U, const void* dU, const void* dmu, int stage, void* E, void* dE)
{
    if (c->prec == M2P_FP64) return Launch<double>::jvp(c->kp, c->B, U, dU, dmu, stage, E, dE, c->stream);
    return Launch<float>::jvp(c->kp, c->B, U, dU, dmu, stage, E, dE, c->stream);
}

struct VjpWork {
    DevBuf GT, DU, FCX, FCY, SC, tmp;
    int alloc(m2p_ctx* c)
    {
        const KParams& K = c->kp;
        const size_t st = (size_t)NF * K.ny * K.pitch * c->esz;
        int rc;
        if ((rc = GT.alloc(st)) || (rc = DU.alloc(st)) || (rc = tmp.alloc(st))) return rc;
        // per-cell x-face sums over the row extended by two ghost columns a side
        if ((rc = FCX.alloc((size_t)K.ny * (K.nx + 4) * NF * c->esz))) return rc;
        if ((rc = FCY.alloc((size_t)(K.ny + 1) * K.nx * 24 * c->esz))) return rc;
        // per target column (row extended by a ghost column a side) the source
        // sums landing level (6 fields), one row up and one row down (4 each)
        return SC.alloc((size_t)K.ny * (K.nx + 2) * 14 * c->esz);
    }
};

// lam_in = (stage transpose at U) (lscale lam) [+ zc z]
hipError_t L_vjp(m2p_ctx* c, VjpWork& w, const void* U, const void* lam, int stage, double dt, void* lam_in,
                 void* gmu, double lscale = 1.0, const void* z = nullptr, double zc = 0.0)
{
    if (c->prec == M2P_FP64)
        return Launch<double>::vjp(c->kp, c->B, U, lam, lscale, stage, dt, w.GT.p, w.DU.p, w.FCX.p, w.FCY.p, w.SC.p,
                                   lam_in, z, zc, gmu, c->stream);
    return Launch<float>::vjp(c->kp, c->B, U, lam, lscale, stage, dt, w.GT.p, w.DU.p, w.FCX.p, w.FCY.p, w.SC.p,
                              lam_in, z, zc, gmu, c->stream);
}

int L_dot(m2p_ctx* c, const void* x, const void* y, double* out)
{
    hipError_t e = c->prec == M2P_FP64 ? Launch<double>::dot(c->kp, x, y, c->mass_part, c->stream)
                                       : Launch<float>::dot(c->kp, x, y, c->mass_part, c->stream);
    HIPCHK(e);
    std::vector<double> part(kMassBlocks);
    HIPCHK(hipMemcpyAsync(part.data(), c->mass_part, kMassBlocks * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    double acc = 0.0;
    for (double v : part) acc += v;
    *out = acc;
    return M2P_OK;
}

int L_loss(m2p_ctx* c, const double* target_dev, void* lam, double* loss)
{
    hipError_t e = c->prec == M2P_FP64
                       ? Launch<double>::loss(c->kp, c->B, c->B.U, target_dev, lam, c->mass_part, c->stream)
                       : Launch<float>::loss(c->kp, c->B, c->B.U, target_dev, lam, c->mass_part, c->stream);
    HIPCHK(e);
    std::vector<double> part(kMassBlocks);
    HIPCHK(hipMemcpyAsync(part.data(), c->mass_part, kMassBlocks * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    double acc = 0.0;
    for (double v : part) acc += v;
    *loss = acc;
    return M2P_OK;
}

static_assert(m2p::kFlagCentralUpwind == M2P_F_CENTRAL_UPWIND, "central-upwind flag bit");
static_assert(m2p::kFlagEarthPressure == M2P_F_EARTH_PRESSURE, "earth-pressure flag bit");
static_assert(m2p::kFlagSmoothFriction == M2P_F_SMOOTH_FRICTION, "smooth-friction flag bit");
static_assert(m2p::kFlagWellBalanced == M2P_F_WELL_BALANCED, "well-balanced flag bit");

// The tangent and adjoint kernels differentiate the Kurganov-Tadmor flux of
// the paper's model.
int flux_unsupported(m2p_ctx* c)
{
    if (c->kp.flags & M2P_F_CENTRAL_UPWIND)
        return m2p::fail(M2P_EINVAL, "the tangent and adjoint kernels differentiate the central (Kurganov-Tadmor) flux");
    if (c->kp.flags & M2P_F_EARTH_PRESSURE)
        return m2p::fail(M2P_EINVAL, "the tangent and adjoint kernels differentiate the model without earth pressure");
    if (c->kp.flags & M2P_F_WELL_BALANCED)
        return m2p::fail(M2P_EINVAL, "the tangent and adjoint kernels differentiate the plain face reconstruction");
    return M2P_OK;
}

int inflow_unsupported(m2p_ctx* c)
{
    if (int rc = flux_unsupported(c)) return rc;
    if (c->kp.nseg > 0 || c->kp.nsseg > 0)
        return m2p::fail(M2P_EINVAL, "the adjoint supports Mode-I (no inflow segments)");
    if (c->kp.rk != 2) return m2p::fail(M2P_EINVAL, "the adjoint differentiates the two-step (Heun) method");
    return M2P_OK;
}

}  // namespace

extern "C" {

int m2p_set_friction_field(m2p_ctx* c, const double* tan_mu)
{
    if (!c || !tan_mu) return fail(M2P_EINVAL, "NULL argument");
    const size_t n = (size_t)c->g.nx * c->g.ny;
    for (size_t k = 0; k < n; k++)
        if (!(tan_mu[k] >= 0.0) || !std::isfinite(tan_mu[k])) return fail(M2P_EINVAL, "bad tan_mu value");
    if (c->p.flags & M2P_F_EARTH_PRESSURE) {
        const int rc = ep_friction_ok(&c->p, tan_mu, n);
        if (rc) return rc;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    if (!c->mu) {
        if (hipMalloc(&c->mu, (size_t)c->g.ny * c->kp.pitch * c->esz) != hipSuccess)
            return fail(M2P_ENOMEM, "friction field allocation failed");
        c->B.mu = c->mu;
    }
    int rc = upload(c, tan_mu, c->mu, 1);
    if (rc) return rc;
    c->kp.has_mu = 1;
    c->dirty = true;
    return M2P_OK;
}

int m2p_set_dt_schedule(m2p_ctx* c, const double* dts, int64_t n)
{
    if (!c || n < 0 || (n > 0 && !dts)) return fail(M2P_EINVAL, "bad argument");
    HIPCHK(hipStreamSynchronize(c->stream));
    static_assert(sizeof(void*) == 8, "64-bit pointers");
    double* dev = nullptr;
    if (n > 0) {
        std::vector<double> v(n);
        for (int64_t k = 0; k < n; k++) {
            if (!(dts[k] > 0.0) || !std::isfinite(dts[k])) return fail(M2P_EINVAL, "time steps must be positive");
            v[k] = dts[k] / c->kp.T;
        }
        if (hipMalloc((void**)&dev, n * 8) != hipSuccess) return fail(M2P_ENOMEM, "schedule allocation failed");
        HIPCHK(hipMemcpy(dev, v.data(), n * 8, hipMemcpyHostToDevice));
    }
    const double* old = nullptr;
    HIPCHK(hipMemcpy(&old, (char*)c->S + offsetof(DevScalars, dt_sched), sizeof(old), hipMemcpyDeviceToHost));
    const long long nn = n;
    HIPCHK(hipMemcpy((char*)c->S + offsetof(DevScalars, dt_sched), &dev, sizeof(dev), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy((char*)c->S + offsetof(DevScalars, n_sched), &nn, sizeof(nn), hipMemcpyHostToDevice));
    if (old) (void)hipFree((void*)old);
    c->dirty = true;
    return M2P_OK;
}

int m2p_loss(m2p_ctx* c, const double* target_h, double* loss)
{
    if (!c || !target_h || !loss) return fail(M2P_EINVAL, "NULL argument");
    if (!c->has_state) return fail(M2P_ESTATE, "no state");
    const size_t n = (size_t)c->g.nx * c->g.ny;
    DevBuf tgt, lam;
    int rc;
    if ((rc = tgt.alloc(n * 8)) || (rc = lam.alloc(c->state_bytes))) return rc;
    HIPCHK(hipMemcpy(tgt.p, target_h, n * 8, hipMemcpyHostToDevice));
    return L_loss(c, (const double*)tgt.p, lam.p, loss);
}

int m2p_loss_noalloc(m2p_ctx* c, const double* target_dev, double* loss_dev)
{
    if (!c || !target_dev || !loss_dev) return fail(M2P_EINVAL, "NULL argument");
    if (!c->has_state) return fail(M2P_ESTATE, "no state");
    if (!c->scratch) return fail(M2P_ESTATE, "scratch array not set up");
    // partials: one per block of the loss kernel (kMassBlocks, checked to fit
    // the scratch array at compile time); no lam output
    hipError_t e = c->prec == M2P_FP64
                       ? Launch<double>::loss(c->kp, c->B, c->B.U, target_dev, nullptr, c->scratch, c->stream)
                       : Launch<float>::loss(c->kp, c->B, c->B.U, target_dev, nullptr, c->scratch, c->stream);
    HIPCHK(e);
    hipLaunchKernelGGL(k_sum_in_order, dim3(1), dim3(64), 0, c->stream, (const double*)c->scratch, kMassBlocks,
                       loss_dev);
    HIPCHK(hipGetLastError());
    return M2P_OK;
}

int m2p_stage_jvp(m2p_ctx* c, int32_t stage, const double* dU, const double* dmu, double* E, double* dE)
{
    if (!c || !dU || !E || !dE || stage < 0 || stage > 1) return fail(M2P_EINVAL, "bad argument");
    int rc = flux_unsupported(c);
    if (rc) return rc;
    rc = ensure_ready(c);
    if (rc) return rc;
    DevBuf ddU, dE_, E_, dmu_;
    if ((rc = ddU.alloc(c->state_bytes)) || (rc = E_.alloc(c->state_bytes)) || (rc = dE_.alloc(c->state_bytes)))
        return rc;
    if ((rc = upload(c, dU, ddU.p, NF))) return rc;
    if (dmu) {
        if ((rc = dmu_.alloc((size_t)c->g.ny * c->kp.pitch * c->esz))) return rc;
        if ((rc = upload(c, dmu, dmu_.p, 1))) return rc;
    }
    HIPCHK(L_jvp(c, c->B.U, ddU.p, dmu_.p, stage, E_.p, dE_.p));
    if ((rc = download(c, E_.p, E, NF))) return rc;
    return download(c, dE_.p, dE, NF);
}

int m2p_stage_vjp(m2p_ctx* c, int32_t stage, const double* lam, double* lam_in, double* gmu)
{
    if (!c || !lam || !lam_in || stage < 0 || stage > 1) return fail(M2P_EINVAL, "bad argument");
    int rc = flux_unsupported(c);
    if (rc) return rc;
    rc = ensure_ready(c);
    if (rc) return rc;
    DevScalars hs;
    if ((rc = read_scalars(c, &hs))) return rc;
    VjpWork w;
    DevBuf l, li, g;
    if ((rc = w.alloc(c)) || (rc = l.alloc(c->state_bytes)) || (rc = li.alloc(c->state_bytes)) ||
        (rc = g.alloc((size_t)c->g.ny * c->kp.pitch * c->esz)))
        return rc;
    if ((rc = upload(c, lam, l.p, NF))) return rc;
    HIPCHK(L_vjp(c, w, c->B.U, l.p, stage, hs.dt, li.p, g.p));
    if ((rc = download(c, li.p, lam_in, NF))) return rc;
    if (gmu) return download(c, g.p, gmu, 1);
    return M2P_OK;
}

int m2p_adjoint_run(m2p_ctx* c, int64_t nsteps, int32_t ckpt_every, const double* target_h, double vol_scale,
                    double* loss, double* grad_mu, double* grad_vol)
{
    if (!c || nsteps < 1 || ckpt_every < 1 || !target_h || !loss || !(vol_scale > 0.0))
        return fail(M2P_EINVAL, "bad argument");
    int rc = inflow_unsupported(c);
    if (rc) return rc;
    if ((rc = ensure_ready(c))) return rc;
    const KParams& K = c->kp;
    const size_t n = (size_t)c->g.nx * c->g.ny, sb = c->state_bytes;
    const int nseg = (int)((nsteps + ckpt_every - 1) / ckpt_every);
    const int seglen = (int)std::min<int64_t>(ckpt_every, nsteps);
    DevBuf ckpt, sck, dts, tapeU, tapeUs, lam, lamv, gmu, tgt, fin, sfin, bscr;
    VjpWork w;
    if ((rc = ckpt.alloc(sb * nseg)) || (rc = sck.alloc(sizeof(DevScalars) * nseg)) ||
        (rc = dts.alloc(8 * nsteps)) || (rc = tapeU.alloc(sb * seglen)) || (rc = tapeUs.alloc(sb * seglen)) ||
        (rc = lam.alloc(sb)) || (rc = lamv.alloc(sb)) ||
        (rc = gmu.alloc((size_t)K.ny * K.pitch * c->esz)) || (rc = tgt.alloc(n * 8)) || (rc = fin.alloc(sb)) ||
        (rc = sfin.alloc(sizeof(DevScalars))) || (rc = w.alloc(c)) ||
        (rc = bscr.alloc(sizeof(double) * (outflow_dt_index(c->B.nmax) + 2))))
        return rc;
    HIPCHK(hipMemcpy(tgt.p, target_h, n * 8, hipMemcpyHostToDevice));
    const hipStream_t st = c->stream;
    // time-step record: dts[0] is the current step's dt; the finalize of
    // step s stores the dt of step s + 1 (the record is switched off again
    // on every way out of this call)
    DevScalars h0;
    if ((rc = read_scalars(c, &h0))) return rc;
    HIPCHK(hipMemcpy(dts.p, &h0.dt, 8, hipMemcpyHostToDevice));
    struct DtLog {
        double* p;
        long long base, n;
    };
    static_assert(offsetof(DevScalars, n_log) == offsetof(DevScalars, dt_log) + offsetof(DtLog, n) &&
                      offsetof(DevScalars, log_base) == offsetof(DevScalars, dt_log) + offsetof(DtLog, base),
                  "time-step record fields");
    const DtLog on{(double*)dts.p, h0.steps, nsteps};
    HIPCHK(hipMemcpy((char*)c->S + offsetof(DevScalars, dt_log), &on, sizeof(on), hipMemcpyHostToDevice));
    struct LogOff {
        DevScalars* S;
        hipStream_t st;
        ~LogOff()
        {
            const DtLog off{nullptr, 0, 0};
            (void)hipStreamSynchronize(st);
            (void)hipMemcpy((char*)S + offsetof(DevScalars, dt_log), &off, sizeof(off), hipMemcpyHostToDevice);
        }
    } log_off{c->S, st};
    // With one segment (ckpt_every >= nsteps) the forward itself writes the
    // tape -- stage 1 reads U^s from tapeU[s] and writes U*^s to tapeUs[s],
    // stage 2 writes U^{s+1} to tapeU[s+1] (the last step to the context's
    // state) -- and the reverse sweep recomputes nothing.  Otherwise the
    // forward keeps a checkpoint per segment (graph-captured chunks between
    // them) and each segment is recomputed before its sweep.
    const bool taped = nseg == 1;
    if (taped) {
        HIPCHK(hipMemcpyAsync(ckpt.p, c->B.U, sb, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(tapeU.p, c->B.U, sb, hipMemcpyDeviceToDevice, st));
        for (int64_t s = 0; s < nsteps; s++) {
            Bufs tb = c->B;
            tb.U = (char*)tapeU.p + sb * s;
            tb.Us = (char*)tapeUs.p + sb * s;
            tb.Uout = s + 1 < nsteps ? (char*)tapeU.p + sb * (s + 1) : c->B.U;
            HIPCHK(step_part(c, tb, 0));
            HIPCHK(step_part(c, tb, 1));
            HIPCHK(step_part(c, tb, 2));
        }
    } else {
        for (int k = 0; k < nseg; k++) {
            HIPCHK(hipMemcpyAsync((char*)ckpt.p + sb * k, c->B.U, sb, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync((char*)sck.p + sizeof(DevScalars) * k, c->S, sizeof(DevScalars),
                                  hipMemcpyDeviceToDevice, st));
            if ((rc = issue_steps(c, std::min<int64_t>(ckpt_every, nsteps - (int64_t)k * ckpt_every)))) return rc;
        }
    }
    DevScalars hs;
    if ((rc = read_scalars(c, &hs)) || (rc = check_status(c, hs))) return rc;
    HIPCHK(hipMemcpyAsync(fin.p, c->B.U, sb, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(sfin.p, c->S, sizeof(DevScalars), hipMemcpyDeviceToDevice, st));
    std::vector<double> hdt(nsteps);
    HIPCHK(hipMemcpyAsync(hdt.data(), dts.p, 8 * nsteps, hipMemcpyDeviceToHost, st));
    if ((rc = L_loss(c, (const double*)tgt.p, lam.p, loss))) return rc;
    // reverse sweep, segment by segment, recomputing each segment's states
    for (int sg = nseg - 1; sg >= 0; sg--) {
        const int64_t n0 = (int64_t)sg * ckpt_every, n1 = std::min<int64_t>(nsteps, n0 + ckpt_every);
        // recompute the segment's states straight into the tapes: stage 1
        // reads U^s from tapeU[s] and writes U*^s to tapeUs[s]; stage 2 writes
        // U^{s+1} to tapeU[s+1].  The last step needs only its stage 1.
        if (!taped) {
            HIPCHK(hipMemcpyAsync(tapeU.p, (char*)ckpt.p + sb * sg, sb, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(c->S, (char*)sck.p + sizeof(DevScalars) * sg, sizeof(DevScalars),
                                  hipMemcpyDeviceToDevice, st));
        }
        for (int64_t s = n0; s < n1 && !taped; s++) {
            Bufs tb = c->B;
            tb.bpart = (double*)bscr.p;  // the recomputation adds nothing to the outflow integrals
            tb.U = (char*)tapeU.p + sb * (s - n0);
            tb.Us = (char*)tapeUs.p + sb * (s - n0);
            HIPCHK(step_part(c, tb, 0));
            if (s + 1 < n1) {
                tb.Uout = (char*)tapeU.p + sb * (s - n0 + 1);
                HIPCHK(step_part(c, tb, 1));
                HIPCHK(step_part(c, tb, 2));
            }
        }
        for (int64_t s = n1 - 1; s >= n0; s--) {
            const double dt = hdt[s];
            const void* Un = (char*)tapeU.p + sb * (s - n0);
            const void* Us = (char*)tapeUs.p + sb * (s - n0);
            // U^{n+1} = (U^n + E(U*)) / 2: half of lambda^{n+1} enters the
            // second stage, and lambda^n = lambda^{n+1} / 2 + (stage-1
            // transpose of the cotangent of U*), summed by the last gather
            HIPCHK(L_vjp(c, w, Us, lam.p, 1, dt, lamv.p, gmu.p, 0.5));              // -> cotangent of U*
            HIPCHK(L_vjp(c, w, Un, lamv.p, 0, dt, lam.p, gmu.p, 1.0, lam.p, 0.5));  // -> lambda^n
        }
    }
    // dL / d(volume scale): the initial state is proportional to the scale
    double dot0 = 0.0;
    if ((rc = L_dot(c, lam.p, ckpt.p, &dot0))) return rc;
    if (grad_vol) *grad_vol = dot0 / vol_scale;
    if (grad_mu && (rc = download(c, gmu.p, grad_mu, 1))) return rc;
    // leave the context at the end of the forward run
    HIPCHK(hipMemcpyAsync(c->B.U, fin.p, sb, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(c->S, sfin.p, sizeof(DevScalars), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return M2P_OK;
}

}  // extern "C"
