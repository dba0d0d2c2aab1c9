// m2p_batch.hip -- C ABI of the batched ensemble (include/m2p.h, m2p_batch_*):
// many independent scenarios of uneven size advanced together.  All states
// live in one ragged SoA arena; one persistent launch per RK stage walks a
// work list of (scenario, strip, row block) items; one finalize workgroup per
// scenario keeps each scenario's own CFL step, time and integrals.  Step
// sequences are captured once into a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "m2p.h"
#include "m2p_host.h"
#include "m2p_launch.h"

using namespace m2p;

struct m2p_batch {
    int prec = M2P_FP32;
    size_t esz = 4;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int nscen = 0;
    std::vector<m2p_grid> g;
    std::vector<KParams> kp;
    std::vector<size_t> u_off, b_off, mu_off, bp_off, wp_off;  // bytes / doubles
    std::vector<int> nmax, nwcap, nw_ref;
    std::vector<char> has_state;
    void* U = nullptr;
    void* Us = nullptr;
    void* b = nullptr;
    void* mu = nullptr;
    DevScalars* S = nullptr;
    double* bpart = nullptr;
    double* wpart = nullptr;
    double* tables = nullptr;
    double* mass_part = nullptr;
    double* staging = nullptr;
    size_t staging_cells = 0;
    size_t u_bytes = 0;
    size_t bp_total = 0;  // doubles of the boundary-slot arena
    void* scen = nullptr;  // ScenDesc<T>[nscen] on the device
    int* work = nullptr;
    int nwork = 0;
    int R = 16, blocks = 0;
    bool buf = true;  // every member's state and DEM below 2 GiB: raw buffer accesses
    bool dirty = true, poisoned = false;
    int graph_chunk = 50;
    hipGraphExec_t gexec = nullptr;
    int gsteps = 0;
};

namespace {

template <typename T>
ScenDesc<T> desc_of(const m2p_batch* B, int i, int R)
{
    ScenDesc<T> d;
    std::memset(&d, 0, sizeof(d));
    d.P = B->kp[i];
    d.U = (T*)((char*)B->U + B->u_off[i]);
    d.Us = (T*)((char*)B->Us + B->u_off[i]);
    d.b = (const T*)((const char*)B->b + B->b_off[i]);
    d.mu = B->kp[i].has_mu ? (const T*)((const char*)B->mu + B->mu_off[i]) : nullptr;
    d.S = B->S + i;
    d.bpart = B->bpart + B->bp_off[i];
    d.wpart = B->wpart + B->wp_off[i];
    d.tables = B->tables;
    d.nmax = B->nmax[i];
    d.nstrips = (B->kp[i].nx + 59) / 60;
    d.nrb = (B->kp[i].ny + R - 1) / R;
    d.nw_ref = B->nw_ref[i];
    return d;
}

void drop_graph(m2p_batch* B)
{
    if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
    B->gexec = nullptr;
    B->gsteps = 0;
}

// Rebuild the device scenario table and the work list for tile height R.
int set_shape(m2p_batch* B, int R, int blocks)
{
    HIPCHK(hipStreamSynchronize(B->stream));
    drop_graph(B);
    std::vector<int> work;
    for (int i = 0; i < B->nscen; i++) {
        const int nstrips = (B->kp[i].nx + 59) / 60, nrb = (B->kp[i].ny + R - 1) / R;
        if ((size_t)nstrips * nrb > (size_t)B->nwcap[i]) return fail(M2P_EINVAL, "tile rows too small");
        for (int w = 0; w < nstrips * nrb; w++) work.push_back((i << 20) | w);
    }
    if (B->work) (void)hipFree(B->work);
    B->work = nullptr;
    HIPCHK(hipMalloc(&B->work, work.size() * sizeof(int)));
    HIPCHK(hipMemcpy(B->work, work.data(), work.size() * sizeof(int), hipMemcpyHostToDevice));
    B->nwork = (int)work.size();
    if (B->prec == M2P_FP64) {
        std::vector<ScenDesc<double>> d;
        for (int i = 0; i < B->nscen; i++) d.push_back(desc_of<double>(B, i, R));
        HIPCHK(hipMemcpy(B->scen, d.data(), d.size() * sizeof(d[0]), hipMemcpyHostToDevice));
    } else {
        std::vector<ScenDesc<float>> d;
        for (int i = 0; i < B->nscen; i++) d.push_back(desc_of<float>(B, i, R));
        HIPCHK(hipMemcpy(B->scen, d.data(), d.size() * sizeof(d[0]), hipMemcpyHostToDevice));
    }
    B->R = R;
    const int full = (B->nwork + 3) / 4;
    B->blocks = blocks > 0 ? std::min(blocks, full) : std::min(full, 2048);
    return M2P_OK;
}

hipError_t part(m2p_batch* B, int p, int mode)
{
    if (B->prec == M2P_FP64)
        return Launch<double>::batch_part((const ScenDesc<double>*)B->scen, B->nscen, B->work, B->nwork, B->R,
                                          B->blocks, B->buf, B->stream, p, mode);
    return Launch<float>::batch_part((const ScenDesc<float>*)B->scen, B->nscen, B->work, B->nwork, B->R, B->blocks,
                                     B->buf, B->stream, p, mode);
}

hipError_t one_step(m2p_batch* B)
{
    for (int p = 0; p < 3; p++) {
        hipError_t e = part(B, p, 0);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

Bufs bufs_of(const m2p_batch* B, int i)
{
    Bufs x;
    std::memset(&x, 0, sizeof(x));
    x.U = (char*)B->U + B->u_off[i];
    x.Us = (char*)B->Us + B->u_off[i];
    x.b = (const char*)B->b + B->b_off[i];
    x.mu = B->kp[i].has_mu ? (const char*)B->mu + B->mu_off[i] : nullptr;
    x.S = B->S + i;
    x.bpart = B->bpart + B->bp_off[i];
    x.wpart = B->wpart + B->wp_off[i];
    x.tables = B->tables;
    x.mass_part = B->mass_part;
    x.nmax = B->nmax[i];
    x.nw_ref = B->nw_ref[i];
    return x;
}

int ensure_ready(m2p_batch* B)
{
    if (B->poisoned) return fail(M2P_ESTATE, "batch poisoned by an earlier device error");
    for (int i = 0; i < B->nscen; i++)
        if (!B->has_state[i]) return fail(M2P_ESTATE, "every scenario needs a state before stepping");
    if (B->dirty) {
        for (int i = 0; i < B->nscen; i++) {
            Bufs x = bufs_of(B, i);
            hipError_t e = B->prec == M2P_FP64 ? Launch<double>::init(B->kp[i], x, B->stream)
                                               : Launch<float>::init(B->kp[i], x, B->stream);
            HIPCHK(e);
        }
        B->dirty = false;
    }
    return M2P_OK;
}

int check_status(m2p_batch* B)
{
    std::vector<DevScalars> hs(B->nscen);
    HIPCHK(hipMemcpyAsync(hs.data(), B->S, hs.size() * sizeof(DevScalars), hipMemcpyDeviceToHost, B->stream));
    HIPCHK(hipStreamSynchronize(B->stream));
    for (int i = 0; i < B->nscen; i++) {
        if (hs[i].status & 1u) {
            B->poisoned = true;
            return fail(M2P_ENONFINITE, "non-finite value in scenario " + std::to_string(i));
        }
        if (hs[i].status & 2u) {
            B->poisoned = true;
            return fail(M2P_EDTFLOOR, "time step floor in scenario " + std::to_string(i));
        }
    }
    return M2P_OK;
}

int run_steps(m2p_batch* B, int64_t n)
{
    int64_t done = 0;
    if (B->graph_chunk > 0 && n >= B->graph_chunk) {
        if (!B->gexec || B->gsteps != B->graph_chunk) {
            drop_graph(B);
            hipGraph_t graph;
            HIPCHK(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
            for (int k = 0; k < B->graph_chunk; k++) {
                hipError_t e = one_step(B);
                if (e != hipSuccess) {
                    (void)hipStreamEndCapture(B->stream, &graph);
                    return hip_fail(e, "kernel launch during graph capture");
                }
            }
            HIPCHK(hipStreamEndCapture(B->stream, &graph));
            hipError_t e = hipGraphInstantiate(&B->gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIPCHK(e);
            B->gsteps = B->graph_chunk;
        }
        for (; done + B->gsteps <= n; done += B->gsteps) HIPCHK(hipGraphLaunch(B->gexec, B->stream));
    }
    for (; done < n; done++) HIPCHK(one_step(B));
    return M2P_OK;
}

}  // namespace

extern "C" {

int m2p_batch_create(m2p_batch** out, int32_t nscen, const m2p_grid* grids, const m2p_params* params,
                     const double* const* dems, const double* const* tan_mu, int32_t prec, void* hip_stream)
{
    if (!out) return fail(M2P_EINVAL, "out is NULL");
    *out = nullptr;
    if (nscen < 1 || nscen > 2047 || !grids || !params || !dems) return fail(M2P_EINVAL, "bad batch arguments");
    for (int i = 0; i < nscen; i++) {
        int rc = validate_scenario(&grids[i], &params[i], prec, dems[i]);
        if (rc) return fail(rc, "scenario " + std::to_string(i) + ": " + m2p_last_error());
        if (params[i].flags & M2P_F_RK3) return fail(M2P_EINVAL, "ensembles run the two-step (Heun) method");
        if (params[i].flags & M2P_F_CENTRAL_UPWIND)
            return fail(M2P_EINVAL, "ensembles run the central (Kurganov-Tadmor) flux");
        if (params[i].flags & M2P_F_EARTH_PRESSURE)
            return fail(M2P_EINVAL, "ensembles run the model without earth pressure");
        if (params[i].flags & M2P_F_WELL_BALANCED)
            return fail(M2P_EINVAL, "ensembles run the plain face reconstruction");
        if (params[i].flags & M2P_F_SMOOTH_FRICTION)
            return fail(M2P_EINVAL, "ensembles run the Coulomb stop-clamp (smooth friction is for gradient checks)");
        if ((size_t)((grids[i].nx + 59) / 60) * (size_t)((grids[i].ny + 3) / 4) >= (1u << 20))
            return fail(M2P_EINVAL, "scenario too large for a batch");
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(M2P_EHIP, "no HIP device");
    m2p_batch* B = new m2p_batch();
    auto bail = [&](int code) {
        m2p_batch_destroy(B);
        return code;
    };
    B->prec = prec;
    B->esz = prec == M2P_FP64 ? 8 : 4;
    B->nscen = nscen;
    if (hip_stream) {
        B->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(M2P_EHIP, "stream creation failed"));
        B->own_stream = true;
    }
    size_t ub = 0, bb = 0, mb = 0, bp = 0, wp = 0, maxcells = 0;
    for (int i = 0; i < nscen; i++) {
        const bool hm = tan_mu && tan_mu[i];
        KParams K = make_kparams(&grids[i], &params[i], hm);
        B->g.push_back(grids[i]);
        B->kp.push_back(K);
        B->u_off.push_back(ub);
        ub += (size_t)NF * K.ny * K.pitch * B->esz;
        B->b_off.push_back(bb);
        bb += (size_t)(K.ny + 2 * BHALO) * K.bpitch * B->esz;
        if ((uint64_t)NF * K.ny * K.pitch * B->esz >= (1ull << 31) ||
            (uint64_t)(K.ny + 2 * BHALO) * K.bpitch * B->esz >= (1ull << 31))
            B->buf = false;
        B->mu_off.push_back(mb);
        if (hm) mb += (size_t)K.ny * K.pitch * B->esz;
        const int nbx = (K.nx + 63) / 64, nby = (K.ny + 3) / 4, nstrips = (K.nx + 59) / 60, nrb = (K.ny + 3) / 4;
        const int nm = std::max(K.nx, K.ny) + 1;  // outflow slots: one per boundary face
        const int nw = std::max(nbx * nby, nstrips * nrb);
        B->nmax.push_back(nm);
        B->nwcap.push_back(nw);
        B->nw_ref.push_back(nbx * nby);
        B->bp_off.push_back(bp);
        bp += outflow_dt_index(nm) + 2;  // keeps each scenario's block 16-byte aligned
        B->wp_off.push_back(wp);
        wp += (size_t)2 * 4 * nw;
        maxcells = std::max(maxcells, (size_t)K.nx * K.ny);
    }
    B->has_state.assign(nscen, 0);
    B->u_bytes = ub;
    B->bp_total = bp;
    if (hipMalloc(&B->U, ub) != hipSuccess || hipMalloc(&B->Us, ub) != hipSuccess ||
        hipMalloc(&B->b, bb) != hipSuccess || hipMalloc(&B->S, nscen * sizeof(DevScalars)) != hipSuccess ||
        hipMalloc(&B->bpart, bp * sizeof(double)) != hipSuccess ||
        hipMalloc(&B->wpart, wp * sizeof(double)) != hipSuccess ||
        hipMalloc(&B->tables, 8 * sizeof(double)) != hipSuccess ||
        hipMalloc(&B->mass_part, 2 * kMassBlocks * sizeof(double)) != hipSuccess ||
        hipMalloc(&B->staging, 6 * maxcells * sizeof(double)) != hipSuccess ||
        hipMalloc(&B->scen, nscen * std::max(sizeof(ScenDesc<double>), sizeof(ScenDesc<float>))) != hipSuccess)
        return bail(fail(M2P_ENOMEM, "batch allocation failed"));
    if (mb && hipMalloc(&B->mu, mb) != hipSuccess) return bail(fail(M2P_ENOMEM, "batch allocation failed"));
    B->staging_cells = maxcells;
    if (hipMemset(B->U, 0, ub) != hipSuccess || hipMemset(B->Us, 0, ub) != hipSuccess ||
        hipMemset(B->bpart, 0, bp * sizeof(double)) != hipSuccess ||
        hipMemset(B->wpart, 0, wp * sizeof(double)) != hipSuccess)
        return bail(fail(M2P_EHIP, "batch initialisation failed"));
    DevScalars hs;
    std::memset(&hs, 0, sizeof(hs));
    hs.t_end = std::numeric_limits<double>::infinity();
    std::vector<DevScalars> hsv(nscen, hs);
    if (hipMemcpy(B->S, hsv.data(), nscen * sizeof(DevScalars), hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(M2P_EHIP, "batch initialisation failed"));
    for (int i = 0; i < nscen; i++) {
        const KParams& K = B->kp[i];
        std::vector<double> bd = padded_dem(K, dems[i], params[i].L);
        hipError_t e;
        if (prec == M2P_FP64) {
            e = hipMemcpy((char*)B->b + B->b_off[i], bd.data(), bd.size() * 8, hipMemcpyHostToDevice);
        } else {
            std::vector<float> bf(bd.begin(), bd.end());
            e = hipMemcpy((char*)B->b + B->b_off[i], bf.data(), bf.size() * 4, hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) return bail(fail(M2P_EHIP, "DEM copy failed"));
        if (K.has_mu) {
            std::vector<double> md((size_t)K.ny * K.pitch, 0.0);
            for (int j = 0; j < K.ny; j++)
                for (int x = 0; x < K.nx; x++) {
                    double v = tan_mu[i][(size_t)j * K.nx + x];
                    if (!(v >= 0.0) || !std::isfinite(v)) return bail(fail(M2P_EINVAL, "bad tan_mu value"));
                    md[(size_t)j * K.pitch + x] = v;
                }
            if (prec == M2P_FP64) {
                e = hipMemcpy((char*)B->mu + B->mu_off[i], md.data(), md.size() * 8, hipMemcpyHostToDevice);
            } else {
                std::vector<float> mf(md.begin(), md.end());
                e = hipMemcpy((char*)B->mu + B->mu_off[i], mf.data(), mf.size() * 4, hipMemcpyHostToDevice);
            }
            if (e != hipSuccess) return bail(fail(M2P_EHIP, "friction copy failed"));
        }
    }
    int rc = set_shape(B, 16, 0);
    if (rc) return bail(rc);
    *out = B;
    return M2P_OK;
}

void m2p_batch_destroy(m2p_batch* B)
{
    if (!B) return;
    if (B->stream) (void)hipStreamSynchronize(B->stream);
    drop_graph(B);
    void* ptrs[] = {B->U, B->Us, B->b, B->mu, B->S, B->bpart, B->wpart, B->tables, B->mass_part, B->staging,
                    B->scen, B->work};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (B->own_stream) (void)hipStreamDestroy(B->stream);
    delete B;
}

int m2p_batch_set_state(m2p_batch* B, int32_t i, int32_t kind, const double* h, const double* phi, const double* vxs,
                        const double* vys, const double* vxf, const double* vyf)
{
    if (!B || i < 0 || i >= B->nscen || !h || !phi) return fail(M2P_EINVAL, "bad argument");
    if (kind != M2P_DEPTH_NORMAL && kind != M2P_DEPTH_VERTICAL) return fail(M2P_EINVAL, "bad depth kind");
    const size_t n = (size_t)B->kp[i].nx * B->kp[i].ny;
    for (size_t k = 0; k < n; k++) {
        if (!std::isfinite(h[k])) return fail(M2P_EINVAL, "thickness must be finite");
        if (h[k] < 0.0) return fail(M2P_ENEGDEPTH, "negative thickness");
        if (!(phi[k] >= 0.0 && phi[k] <= 1.0)) return fail(M2P_EINVAL, "solid fraction outside [0, 1]");
    }
    const double* v[4] = {vxs, vys, vxf, vyf};
    std::vector<double> f(6 * n, 0.0);
    std::memcpy(f.data(), h, n * 8);
    std::memcpy(f.data() + n, phi, n * 8);
    int has_v = 0;
    for (int q = 0; q < 4; q++)
        if (v[q]) {
            for (size_t k = 0; k < n; k++)
                if (!std::isfinite(v[q][k])) return fail(M2P_EINVAL, "non-finite velocity");
            std::memcpy(f.data() + (2 + q) * n, v[q], n * 8);
            has_v = 1;
        }
    HIPCHK(hipMemcpyAsync(B->staging, f.data(), 6 * n * 8, hipMemcpyHostToDevice, B->stream));
    Bufs x = bufs_of(B, i);
    hipError_t e = B->prec == M2P_FP64
                       ? Launch<double>::set_state(B->kp[i], x, B->staging, kind == M2P_DEPTH_VERTICAL, has_v, B->stream)
                       : Launch<float>::set_state(B->kp[i], x, B->staging, kind == M2P_DEPTH_VERTICAL, has_v, B->stream);
    HIPCHK(e);
    HIPCHK(hipStreamSynchronize(B->stream));
    B->has_state[i] = 1;
    B->dirty = true;
    return M2P_OK;
}

int m2p_batch_get_state_raw(m2p_batch* B, int32_t i, double* U)
{
    if (!B || i < 0 || i >= B->nscen || !U) return fail(M2P_EINVAL, "bad argument");
    const KParams& K = B->kp[i];
    const size_t n = (size_t)K.nx * K.ny, tot = (size_t)NF * K.ny * K.pitch;
    HIPCHK(hipStreamSynchronize(B->stream));
    std::vector<double> h(tot);
    if (B->prec == M2P_FP64) {
        HIPCHK(hipMemcpy(h.data(), (char*)B->U + B->u_off[i], tot * 8, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> f(tot);
        HIPCHK(hipMemcpy(f.data(), (char*)B->U + B->u_off[i], tot * 4, hipMemcpyDeviceToHost));
        std::copy(f.begin(), f.end(), h.begin());
    }
    for (int k = 0; k < NF; k++)
        for (int j = 0; j < K.ny; j++)
            std::memcpy(&U[k * n + (size_t)j * K.nx], &h[((size_t)k * K.ny + j) * K.pitch], K.nx * 8);
    return M2P_OK;
}

int m2p_batch_get_fields(m2p_batch* B, int32_t i, double* h, double* phi, double* vxs, double* vys, double* vxf,
                         double* vyf)
{
    if (!B || i < 0 || i >= B->nscen) return fail(M2P_EINVAL, "bad argument");
    const KParams& K = B->kp[i];
    const size_t n = (size_t)K.nx * K.ny;
    Bufs x = bufs_of(B, i);
    hipError_t e = B->prec == M2P_FP64 ? Launch<double>::get_fields(K, x, B->staging, B->stream)
                                       : Launch<float>::get_fields(K, x, B->staging, B->stream);
    HIPCHK(e);
    std::vector<double> f(6 * n);
    HIPCHK(hipMemcpyAsync(f.data(), B->staging, 6 * n * 8, hipMemcpyDeviceToHost, B->stream));
    HIPCHK(hipStreamSynchronize(B->stream));
    double* o[6] = {h, phi, vxs, vys, vxf, vyf};
    for (int q = 0; q < 6; q++)
        if (o[q]) std::memcpy(o[q], f.data() + q * n, n * 8);
    return M2P_OK;
}

int m2p_batch_get_diag(m2p_batch* B, int32_t i, m2p_diag* d)
{
    if (!B || i < 0 || i >= B->nscen || !d) return fail(M2P_EINVAL, "bad argument");
    std::memset(d, 0, sizeof(*d));
    DevScalars hs;
    HIPCHK(hipMemcpyAsync(&hs, B->S + i, sizeof(hs), hipMemcpyDeviceToHost, B->stream));
    const KParams& K = B->kp[i];
    Bufs x = bufs_of(B, i);
    hipError_t e = B->prec == M2P_FP64 ? Launch<double>::mass(K, x, B->stream) : Launch<float>::mass(K, x, B->stream);
    HIPCHK(e);
    std::vector<double> part(2 * kMassBlocks);
    HIPCHK(hipMemcpyAsync(part.data(), B->mass_part, part.size() * 8, hipMemcpyDeviceToHost, B->stream));
    HIPCHK(hipStreamSynchronize(B->stream));
    double ms = 0.0, mf = 0.0;
    for (int q = 0; q < kMassBlocks; q++) {
        ms += part[2 * q];
        mf += part[2 * q + 1];
    }
    const double scale = K.H * K.L * K.L * K.dxi * K.deta;
    d->mass_s = ms * scale;
    d->mass_f = mf * scale;
    d->t = hs.t * K.T;
    d->dt_last = hs.dt_last * K.T;
    d->dt_next = hs.dt * K.T;
    d->in_s = hs.in_s;
    d->in_f = hs.in_f;
    const int rc = outflow_volumes(B->bpart + B->bp_off[i], B->nmax[i], K.nx, K.ny, K, B->stream, &d->out_s,
                                   &d->out_f);
    if (rc) return rc;
    d->steps = hs.steps;
    d->clamp_count = (int64_t)hs.clamps;
    d->status = (int32_t)hs.status;
    return M2P_OK;
}

int m2p_batch_set_tile(m2p_batch* B, int32_t rows, int32_t blocks)
{
    if (!B || rows < 4 || rows > 4096 || blocks < 0) return fail(M2P_EINVAL, "bad tile arguments");
    return set_shape(B, rows, blocks);
}

int m2p_batch_set_graph(m2p_batch* B, int32_t chunk)
{
    if (!B || chunk < 0) return fail(M2P_EINVAL, "bad argument");
    HIPCHK(hipStreamSynchronize(B->stream));
    drop_graph(B);
    B->graph_chunk = chunk;
    return M2P_OK;
}

int m2p_batch_run(m2p_batch* B, int64_t nsteps)
{
    if (!B || nsteps < 0) return fail(M2P_EINVAL, "bad argument");
    int rc = ensure_ready(B);
    if (rc) return rc;
    return run_steps(B, nsteps);
}

int m2p_batch_synchronize(m2p_batch* B)
{
    if (!B) return fail(M2P_EINVAL, "NULL batch");
    HIPCHK(hipStreamSynchronize(B->stream));
    return check_status(B);
}

// Time a few steps per candidate tile shape on the batch itself (states and
// scalars are saved first and restored after every trial) and keep the
// fastest.  Candidates: tile rows 8, 16, 32, 64 x persistent grids of 1024,
// 2048, 4096 workgroups and one workgroup per four work items.
int m2p_batch_autotune(m2p_batch* B, int32_t trial_steps, int32_t* rows_out, int32_t* blocks_out, double* ms_out)
{
    if (!B || trial_steps < 1) return fail(M2P_EINVAL, "bad argument");
    int rc = ensure_ready(B);
    if (rc) return rc;
    void* backup = nullptr;
    DevScalars* sback = nullptr;
    double* bback = nullptr;
    const size_t bbytes = B->bp_total * sizeof(double);
    if (hipMalloc(&backup, B->u_bytes) != hipSuccess || hipMalloc(&sback, B->nscen * sizeof(DevScalars)) != hipSuccess ||
        hipMalloc(&bback, bbytes) != hipSuccess) {
        if (backup) (void)hipFree(backup);
        if (sback) (void)hipFree(sback);
        return fail(M2P_ENOMEM, "autotune backup allocation failed");
    }
    HIPCHK(hipMemcpyAsync(backup, B->U, B->u_bytes, hipMemcpyDeviceToDevice, B->stream));
    HIPCHK(hipMemcpyAsync(sback, B->S, B->nscen * sizeof(DevScalars), hipMemcpyDeviceToDevice, B->stream));
    HIPCHK(hipMemcpyAsync(bback, B->bpart, bbytes, hipMemcpyDeviceToDevice, B->stream));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const int saved_chunk = B->graph_chunk;
    B->graph_chunk = 0;
    double best = 1e300;
    int bestR = B->R, bestB = B->blocks;
    for (int R : {8, 16, 32, 64}) {
        for (int blocks : {1024, 2048, 4096, 0x7fffffff}) {
            rc = set_shape(B, R, blocks);
            if (rc) break;
            HIPCHK(one_step(B));  // warm
            HIPCHK(hipEventRecord(e0, B->stream));
            for (int k = 0; k < trial_steps; k++) HIPCHK(one_step(B));
            HIPCHK(hipEventRecord(e1, B->stream));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                bestR = R;
                bestB = B->blocks;
            }
            HIPCHK(hipMemcpyAsync(B->U, backup, B->u_bytes, hipMemcpyDeviceToDevice, B->stream));
            HIPCHK(hipMemcpyAsync(B->S, sback, B->nscen * sizeof(DevScalars), hipMemcpyDeviceToDevice, B->stream));
            HIPCHK(hipMemcpyAsync(B->bpart, bback, bbytes, hipMemcpyDeviceToDevice, B->stream));
        }
        if (rc) break;
    }
    HIPCHK(hipStreamSynchronize(B->stream));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(backup);
    (void)hipFree(sback);
    (void)hipFree(bback);
    B->graph_chunk = saved_chunk;
    int rc2 = set_shape(B, bestR, bestB);
    if (rc) return rc;
    if (rc2) return rc2;
    if (rows_out) *rows_out = bestR;
    if (blocks_out) *blocks_out = bestB;
    if (ms_out) *ms_out = best / trial_steps;
    return M2P_OK;
}

int m2p_batch_info(m2p_batch* B, int32_t* nscen, int64_t* cells, int32_t* rows, int32_t* blocks, int32_t* nwork)
{
    if (!B) return fail(M2P_EINVAL, "NULL batch");
    int64_t c = 0;
    for (const KParams& K : B->kp) c += (int64_t)K.nx * K.ny;
    if (nscen) *nscen = B->nscen;
    if (cells) *cells = c;
    if (rows) *rows = B->R;
    if (blocks) *blocks = B->blocks;
    if (nwork) *nwork = B->nwork;
    return M2P_OK;
}

}  // extern "C"
