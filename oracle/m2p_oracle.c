/*
 * m2p_oracle.c -- plain, slow FP64 CPU oracle for the two-phase (grain + fluid)
 * depth-integrated shallow-flow step of MoSES_2PDF (Ko, Chen, Wong, Tai).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the tests, the smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the HIP path.
 *
 * Everything is double precision, one loop nest per sub-step, written in the
 * notation of the paper's Appendix A (model equations) and Sect. 2.2
 * (numerics): an anti-diffusive non-oscillatory central scheme (Kurganov and
 * Tadmor 2000) with minmod-limited linear reconstruction, advanced by the
 * two-step modified Euler method (Heun, second-order Runge-Kutta) with a
 * CFL-limited time step.  Readings chosen where the paper is silent are marked
 * "reading:"; the same readings are followed by the HIP path.  Options beside
 * the paper's choices (params.flags): the three-stage SSP Runge-Kutta method,
 * the central-upwind face flux with one-sided speeds, Savage-Hutter
 * earth-pressure coefficients from the internal friction angle, a smooth
 * (regularised) Coulomb friction for finite-difference checks of gradients,
 * and a well-balanced hydrostatic reconstruction of the face states.
 *
 * Units: SI at the interface; inside, the shallow scaling X, Y, b ~ L,
 * h ~ H, v ~ sqrt(g L), t ~ sqrt(L / g), aspect ratio eps = H / L.
 * Conserved state per cell (6 fields): m^s = J h^s, p^s = J h^s v^s (X and Y),
 * m^f = J h^f, p^f = J h^f v^f (the momentum vectors q^s, q^f of the paper's
 * momentum balances); m = J h is the vertical thickness over H.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define NF 6 /* ms, pxs, pys, mf, pxf, pyf */
#define HALO 2

typedef struct {
    int32_t nx, ny;
    double dx, dy;
    double delta_b_deg, c_d, inv_n_r, theta_b, rho_s, rho_f, cfl;
    double L, H, chi, g, m_dry, a_min;
    int32_t bc[4]; /* W, E, S, N: 0 transmissive, 1 closed wall */
    int32_t flags; /* bit 0: fluid interphase pressure weighted by phi^f as printed;
                      bit 1: three-stage third-order SSP Runge-Kutta instead of Heun;
                      bit 2: central-upwind face flux (one-sided local speeds);
                      bit 3: Savage-Hutter earth-pressure coefficients on the solid pressure;
                      bit 4: smooth Coulomb friction with regularisation speed v_eps;
                      bit 5: well-balanced hydrostatic reconstruction (Mode-II inflow only as ghost states) */
    double delta_int_deg; /* internal friction angle (used with bit 3) */
    double v_eps;         /* m/s (used with bit 4) */
} ora_params;

typedef struct {
    int32_t side, i0, ncells, nt;
    const double *t, *Q, *phi;
} ora_inflow_in;

typedef struct {
    int side, i0, ncells, nt;
    double *t, *Q, *phi;
} inflow_seg;

/* Mode-II segment given as the state of the inflowing flow (hydrographs of
 * vertical thickness h in m, solid fraction, inward speed v in m/s). */
typedef struct {
    int32_t side, i0, ncells, nt;
    const double *t, *h, *phi, *v;
} ora_state_in;

typedef struct {
    int side, i0, ncells, nt;
    double *t, *h, *phi, *v;
} state_seg;

/* Geometry of the basal surface at one cell (Appendix A, O_xi-eta-zeta frame). */
typedef struct {
    double bX, bY;          /* DEM slopes */
    double J, c;            /* J_b = det Omega_b, c = n_Z */
    double nX, nY, nZ;      /* unit normal */
    double A11, A12, A21, A22; /* (A_ij) = Omega_b^{-1}, upper 2x2 block */
} geo_t;

typedef struct {
    ora_params p;
    int nx, ny, px, py; /* padded sizes */
    /* derived, dimensionless */
    double eps, alpha, dxi, deta, md, eps_chi, tan_d, T, V;
    double *b;           /* padded DEM / L */
    double *tan_mu;      /* per-cell tan(delta_b) or NULL */
    double *U;           /* state, 6 * nx * ny */
    /* work arrays */
    double *Ue;          /* padded state */
    geo_t *G;            /* padded geometry (ring 1 used) */
    double *dnx, *dny;   /* d n / d xi, d n / d eta (3 each) per interior cell */
    double *HX, *HY;     /* face fluxes */
    double *HXcL, *HXcR, *HYcL, *HYcR; /* well-balanced option: pressure corrections of the face's left / right cell */
    double *Us, *Uss;
    inflow_seg *seg;
    int nseg;
    state_seg *sseg;
    int nsseg;
    double t;
    int64_t steps, clamps;
    double in_s, in_f, out_s, out_f;
    double bflux[3][2]; /* per stage, per phase: net outward boundary mass flux rate */
    double last_dt;
    double *dt_sched;   /* optional prescribed time steps (dimensionless) */
    int64_t n_sched;
    double cos2_int;    /* cos^2 of the internal friction angle (earth pressure) */
    double *Kx, *Ky;    /* padded earth-pressure coefficients of the stage input */
} ora_sim;

/* ---------------------------------------------------------------- helpers */

#define PIDX(o, i, j) ((size_t)((j) + HALO) * (size_t)(o)->px + (size_t)((i) + HALO))
#define CIDX(o, i, j) ((size_t)(j) * (size_t)(o)->nx + (size_t)(i))

static double minmod(double a, double b)
{
    if (a > 0.0 && b > 0.0) return a < b ? a : b;
    if (a < 0.0 && b < 0.0) return a > b ? a : b;
    return 0.0;
}

/* reading: continuous desingularisation of a ratio num/den for den -> 0
 * (Kurganov and Petrova 2007): 2 den num / (den^2 + max(den^2, md^2)),
 * exactly num/den when den >= md. */
static double desing(double num, double den, double md)
{
    double d2 = den * den;
    double m2 = md * md;
    return (2.0 * den * num) / (d2 + (d2 > m2 ? d2 : m2));
}

static void *xcalloc(size_t n, size_t s) { return calloc(n ? n : 1, s); }

/* ------------------------------------------------------- setup and state */

int ora_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* reading: the DEM is continued outside the domain by linear extrapolation,
 * first along Y for every column, then along X for every (extended) row. */
static void extend_dem(ora_sim *o, const double *dem)
{
    int nx = o->nx, ny = o->ny;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) o->b[PIDX(o, i, j)] = dem[CIDX(o, i, j)] / o->p.L;
    for (int i = 0; i < nx; i++) {
        double b0 = o->b[PIDX(o, i, 0)], b1 = o->b[PIDX(o, i, 1)];
        double bn = o->b[PIDX(o, i, ny - 1)], bm = o->b[PIDX(o, i, ny - 2)];
        for (int k = 1; k <= HALO; k++) {
            o->b[PIDX(o, i, -k)] = b0 + (double)(-k) * (b1 - b0);
            o->b[PIDX(o, i, ny - 1 + k)] = bn + (double)k * (bn - bm);
        }
    }
    for (int j = -HALO; j < ny + HALO; j++) {
        double b0 = o->b[PIDX(o, 0, j)], b1 = o->b[PIDX(o, 1, j)];
        double bn = o->b[PIDX(o, nx - 1, j)], bm = o->b[PIDX(o, nx - 2, j)];
        for (int k = 1; k <= HALO; k++) {
            o->b[PIDX(o, -k, j)] = b0 + (double)(-k) * (b1 - b0);
            o->b[PIDX(o, nx - 1 + k, j)] = bn + (double)k * (bn - bm);
        }
    }
}

/* Basal geometry from the DEM.  The paper builds O_xi-eta-zeta on the DEM with
 * the xi, eta axes projecting onto X, Y (Sect. 2.1) and cites Omega_b only.
 * reading: covariant tangents g_xi = (1, 0, b_X), g_eta = (0, 1, b_Y), unit
 * normal n = (-b_X, -b_Y, 1)/s with s = sqrt(1 + b_X^2 + b_Y^2), Omega_b =
 * [g_xi g_eta n] (columns).  Then J_b = det Omega_b = s, c = n_Z = 1/s, and the
 * upper 2x2 block of Omega_b^{-1} is the inverse surface metric.  b_X, b_Y are
 * central differences. */
static void geometry_at(const ora_sim *o, int i, int j, geo_t *g)
{
    const double *b = o->b;
    double bX = (b[PIDX(o, i + 1, j)] - b[PIDX(o, i - 1, j)]) / (2.0 * o->dxi);
    double bY = (b[PIDX(o, i, j + 1)] - b[PIDX(o, i, j - 1)]) / (2.0 * o->deta);
    double s = sqrt(1.0 + bX * bX + bY * bY);
    g->bX = bX;
    g->bY = bY;
    g->J = s;
    g->c = 1.0 / s;
    g->nX = -bX / s;
    g->nY = -bY / s;
    g->nZ = 1.0 / s;
    g->A11 = (1.0 + bY * bY) / (s * s);
    g->A12 = -bX * bY / (s * s);
    g->A21 = g->A12;
    g->A22 = (1.0 + bX * bX) / (s * s);
}

ora_sim *ora_create(const ora_params *p, const double *dem, const double *tan_mu)
{
    if (p->nx < 2 || p->ny < 2) return NULL;
    if ((p->flags & 16) && !(p->v_eps > 0.0)) return NULL;
    if ((p->flags & 32) && (p->flags & 8)) return NULL; /* not with earth pressure */
    if (p->flags & 8) {
        /* earth pressure needs delta_b <= delta_int < 90 deg everywhere */
        if (!(p->delta_int_deg >= 0.0 && p->delta_int_deg < 90.0) || p->delta_b_deg > p->delta_int_deg) return NULL;
        if (tan_mu) {
            double ti = tan(p->delta_int_deg * M_PI / 180.0);
            for (size_t k = 0; k < (size_t)p->nx * p->ny; k++)
                if (!(tan_mu[k] <= ti)) return NULL;
        }
    }
    ora_sim *o = (ora_sim *)xcalloc(1, sizeof(ora_sim));
    o->p = *p;
    o->nx = p->nx;
    o->ny = p->ny;
    o->px = p->nx + 2 * HALO;
    o->py = p->ny + 2 * HALO;
    o->eps = p->H / p->L;
    o->alpha = p->rho_f / p->rho_s;
    o->dxi = p->dx / p->L;
    o->deta = p->dy / p->L;
    o->md = p->m_dry / p->H;
    o->eps_chi = pow(o->eps, p->chi);
    o->tan_d = tan(p->delta_b_deg * M_PI / 180.0);
    o->T = sqrt(p->L / p->g);     /* time scale */
    o->V = sqrt(p->g * p->L);     /* velocity scale */
    size_t npad = (size_t)o->px * o->py, nc = (size_t)o->nx * o->ny;
    o->b = (double *)xcalloc(npad, sizeof(double));
    o->U = (double *)xcalloc(NF * nc, sizeof(double));
    o->Us = (double *)xcalloc(NF * nc, sizeof(double));
    o->Uss = (double *)xcalloc(NF * nc, sizeof(double));
    o->Ue = (double *)xcalloc(NF * npad, sizeof(double));
    o->G = (geo_t *)xcalloc(npad, sizeof(geo_t));
    o->dnx = (double *)xcalloc(3 * nc, sizeof(double));
    o->dny = (double *)xcalloc(3 * nc, sizeof(double));
    o->HX = (double *)xcalloc(NF * (size_t)(o->nx + 1) * o->ny, sizeof(double));
    o->HY = (double *)xcalloc(NF * (size_t)o->nx * (o->ny + 1), sizeof(double));
    if (p->flags & 32) {
        o->HXcL = (double *)xcalloc(NF * (size_t)(o->nx + 1) * o->ny, sizeof(double));
        o->HXcR = (double *)xcalloc(NF * (size_t)(o->nx + 1) * o->ny, sizeof(double));
        o->HYcL = (double *)xcalloc(NF * (size_t)o->nx * (o->ny + 1), sizeof(double));
        o->HYcR = (double *)xcalloc(NF * (size_t)o->nx * (o->ny + 1), sizeof(double));
    }
    if (tan_mu) {
        o->tan_mu = (double *)xcalloc(nc, sizeof(double));
        memcpy(o->tan_mu, tan_mu, nc * sizeof(double));
    }
    if (p->flags & 8) {
        double ci = cos(p->delta_int_deg * M_PI / 180.0);
        o->cos2_int = ci * ci;
        o->Kx = (double *)xcalloc(npad, sizeof(double));
        o->Ky = (double *)xcalloc(npad, sizeof(double));
    }
    extend_dem(o, dem);
    /* static geometry on the interior plus one ghost ring */
    for (int j = -1; j <= o->ny; j++)
        for (int i = -1; i <= o->nx; i++) geometry_at(o, i, j, &o->G[PIDX(o, i, j)]);
    /* d n / d xi and d n / d eta at interior cells, central differences */
    for (int j = 0; j < o->ny; j++)
        for (int i = 0; i < o->nx; i++) {
            const geo_t *e = &o->G[PIDX(o, i + 1, j)], *w = &o->G[PIDX(o, i - 1, j)];
            const geo_t *nn = &o->G[PIDX(o, i, j + 1)], *s = &o->G[PIDX(o, i, j - 1)];
            size_t c = CIDX(o, i, j);
            o->dnx[3 * c + 0] = (e->nX - w->nX) / (2.0 * o->dxi);
            o->dnx[3 * c + 1] = (e->nY - w->nY) / (2.0 * o->dxi);
            o->dnx[3 * c + 2] = (e->nZ - w->nZ) / (2.0 * o->dxi);
            o->dny[3 * c + 0] = (nn->nX - s->nX) / (2.0 * o->deta);
            o->dny[3 * c + 1] = (nn->nY - s->nY) / (2.0 * o->deta);
            o->dny[3 * c + 2] = (nn->nZ - s->nZ) / (2.0 * o->deta);
        }
    return o;
}

void ora_destroy(ora_sim *o)
{
    if (!o) return;
    free(o->b); free(o->U); free(o->Us); free(o->Uss); free(o->Ue); free(o->G);
    free(o->dnx); free(o->dny); free(o->HX); free(o->HY); free(o->tan_mu); free(o->dt_sched);
    free(o->HXcL); free(o->HXcR); free(o->HYcL); free(o->HYcR);
    free(o->Kx); free(o->Ky);
    for (int k = 0; k < o->nseg; k++) { free(o->seg[k].t); free(o->seg[k].Q); free(o->seg[k].phi); }
    free(o->seg);
    for (int k = 0; k < o->nsseg; k++) { free(o->sseg[k].t); free(o->sseg[k].h); free(o->sseg[k].phi); free(o->sseg[k].v); }
    free(o->sseg);
    free(o);
}

/* Initial state from SI fields.  ``vertical`` != 0: h holds vertical thickness;
 * otherwise the bed-normal thickness h of the paper (vertical = J h). */
int ora_set_state_si(ora_sim *o, int vertical, const double *h, const double *phi_s,
                     const double *vxs, const double *vys, const double *vxf, const double *vyf)
{
    size_t nc = (size_t)o->nx * o->ny;
    for (int j = 0; j < o->ny; j++)
        for (int i = 0; i < o->nx; i++) {
            size_t c = CIDX(o, i, j);
            double J = o->G[PIDX(o, i, j)].J;
            double hv = vertical ? h[c] / o->p.H : J * h[c] / o->p.H;
            double ph = phi_s[c];
            if (!(hv >= 0.0) || !(ph >= 0.0 && ph <= 1.0)) return -1;
            double ms = ph * hv, mf = (1.0 - ph) * hv;
            o->U[0 * nc + c] = ms;
            o->U[1 * nc + c] = vxs ? ms * vxs[c] / o->V : 0.0;
            o->U[2 * nc + c] = vys ? ms * vys[c] / o->V : 0.0;
            o->U[3 * nc + c] = mf;
            o->U[4 * nc + c] = vxf ? mf * vxf[c] / o->V : 0.0;
            o->U[5 * nc + c] = vyf ? mf * vyf[c] / o->V : 0.0;
        }
    return 0;
}

void ora_set_state_raw(ora_sim *o, const double *U) { memcpy(o->U, U, NF * (size_t)o->nx * o->ny * sizeof(double)); }
void ora_get_state_raw(const ora_sim *o, double *U) { memcpy(U, o->U, NF * (size_t)o->nx * o->ny * sizeof(double)); }
void ora_set_time(ora_sim *o, double t_si) { o->t = t_si / o->T; }

int ora_set_inflow(ora_sim *o, const ora_inflow_in *in, int n)
{
    /* the well-balanced option takes Mode-II inflow as ghost states only (a
     * prescribed face flux has no reconstructed state to balance) */
    if ((o->p.flags & 32) && n > 0) return -1;
    o->seg = (inflow_seg *)xcalloc((size_t)n, sizeof(inflow_seg));
    o->nseg = n;
    for (int k = 0; k < n; k++) {
        inflow_seg *s = &o->seg[k];
        s->side = in[k].side; s->i0 = in[k].i0; s->ncells = in[k].ncells; s->nt = in[k].nt;
        int len = (s->side < 2) ? o->ny : o->nx;
        if (s->nt < 1 || s->ncells < 1 || s->i0 < 0 || s->i0 + s->ncells > len) return -1;
        s->t = (double *)xcalloc((size_t)s->nt, sizeof(double));
        s->Q = (double *)xcalloc((size_t)s->nt, sizeof(double));
        s->phi = (double *)xcalloc((size_t)s->nt, sizeof(double));
        memcpy(s->t, in[k].t, (size_t)s->nt * sizeof(double));
        memcpy(s->Q, in[k].Q, (size_t)s->nt * sizeof(double));
        memcpy(s->phi, in[k].phi, (size_t)s->nt * sizeof(double));
    }
    return 0;
}

/* Replace the state-inflow segments.  Segments must lie on their side and
 * must not share a boundary cell with a flux-inflow segment or each other. */
int ora_set_inflow_states(ora_sim *o, const ora_state_in *in, int n)
{
    for (int k = 0; k < o->nsseg; k++) { free(o->sseg[k].t); free(o->sseg[k].h); free(o->sseg[k].phi); free(o->sseg[k].v); }
    free(o->sseg);
    o->sseg = (state_seg *)xcalloc((size_t)n, sizeof(state_seg));
    o->nsseg = n;
    for (int k = 0; k < n; k++) {
        state_seg *s = &o->sseg[k];
        s->side = in[k].side; s->i0 = in[k].i0; s->ncells = in[k].ncells; s->nt = in[k].nt;
        int len = (s->side < 2) ? o->ny : o->nx;
        if (s->side < 0 || s->side > 3 || s->nt < 1 || s->ncells < 1 || s->i0 < 0 || s->i0 + s->ncells > len) return -1;
        for (int q = 0; q < o->nseg; q++)
            if (o->seg[q].side == s->side && s->i0 < o->seg[q].i0 + o->seg[q].ncells && o->seg[q].i0 < s->i0 + s->ncells)
                return -1;
        for (int q = 0; q < k; q++)
            if (o->sseg[q].side == s->side && s->i0 < o->sseg[q].i0 + o->sseg[q].ncells && o->sseg[q].i0 < s->i0 + s->ncells)
                return -1;
        s->t = (double *)xcalloc((size_t)s->nt, sizeof(double));
        s->h = (double *)xcalloc((size_t)s->nt, sizeof(double));
        s->phi = (double *)xcalloc((size_t)s->nt, sizeof(double));
        s->v = (double *)xcalloc((size_t)s->nt, sizeof(double));
        memcpy(s->t, in[k].t, (size_t)s->nt * sizeof(double));
        memcpy(s->h, in[k].h, (size_t)s->nt * sizeof(double));
        memcpy(s->phi, in[k].phi, (size_t)s->nt * sizeof(double));
        memcpy(s->v, in[k].v, (size_t)s->nt * sizeof(double));
    }
    return 0;
}

/* ---------------------------------------------------------- boundaries */

/* Index map for a ghost cell.  Transmissive (the paper's non-reflecting
 * boundary, Sect. 3.1.2): copy the edge cell.  Closed wall: mirror, with the
 * normal momentum of both phases negated. */
static int map_index(int i, int n, int bc_lo, int bc_hi, int *flip)
{
    if (i < 0) {
        if (bc_lo == 1) { *flip ^= 1; return -1 - i; }
        return 0;
    }
    if (i >= n) {
        if (bc_hi == 1) { *flip ^= 1; return 2 * n - 1 - i; }
        return n - 1;
    }
    return i;
}

static double interp(const double *t, const double *y, int n, double tau);

/* reading (literal Mode-II, Sect. 3.1.2 Stage 0): the ghost cells outside a
 * state-inflow segment hold the inflowing flow given by the hydrographs at the
 * stage time: vertical thickness h (m = h / H), solid fraction phi, both
 * phases moving along the inward boundary normal with speed v; the boundary
 * face flux is then the scheme's own central flux. */
static void ghost_state(const ora_sim *o, const state_seg *s, double tau_nd, double u[NF], double *m_out,
                        double *v_out)
{
    double tau = tau_nd * o->T;
    double m = interp(s->t, s->h, s->nt, tau) / o->p.H;
    double ph = interp(s->t, s->phi, s->nt, tau);
    double v = interp(s->t, s->v, s->nt, tau) / o->V;
    if (m_out) *m_out = m;
    if (v_out) *v_out = v;
    double ex = s->side == 0 ? 1.0 : (s->side == 1 ? -1.0 : 0.0);
    double ey = s->side == 2 ? 1.0 : (s->side == 3 ? -1.0 : 0.0);
    double ms = ph * m, mf = (1.0 - ph) * m;
    u[0] = ms;
    u[1] = ms * v * ex;
    u[2] = ms * v * ey;
    u[3] = mf;
    u[4] = mf * v * ex;
    u[5] = mf * v * ey;
}

static void extend_state(ora_sim *o, const double *U, double tau)
{
    size_t nc = (size_t)o->nx * o->ny;
    for (int j = -HALO; j < o->ny + HALO; j++)
        for (int i = -HALO; i < o->nx + HALO; i++) {
            int fx = 0, fy = 0;
            int ii = map_index(i, o->nx, o->p.bc[0], o->p.bc[1], &fx);
            int jj = map_index(j, o->ny, o->p.bc[2], o->p.bc[3], &fy);
            size_t c = CIDX(o, ii, jj), q = PIDX(o, i, j);
            size_t np = (size_t)o->px * o->py;
            for (int k = 0; k < NF; k++) {
                double v = U[k * nc + c];
                if ((k == 1 || k == 4) && fx) v = -v;
                if ((k == 2 || k == 5) && fy) v = -v;
                o->Ue[k * np + q] = v;
            }
        }
    size_t np = (size_t)o->px * o->py;
    for (int sg = 0; sg < o->nsseg; sg++) {
        const state_seg *s = &o->sseg[sg];
        double u[NF];
        ghost_state(o, s, tau, u, NULL, NULL);
        for (int k = s->i0; k < s->i0 + s->ncells; k++)
            for (int l = 1; l <= HALO; l++) {
                int i = s->side == 0 ? -l : (s->side == 1 ? o->nx - 1 + l : k);
                int j = s->side == 2 ? -l : (s->side == 3 ? o->ny - 1 + l : k);
                for (int f = 0; f < NF; f++) o->Ue[f * np + PIDX(o, i, j)] = u[f];
            }
    }
}

/* ------------------------------------------------------- earth pressure */

/* Savage-Hutter earth-pressure coefficients (Savage and Hutter 1989; the
 * two-dimensional form of Hutter et al. 1993), from the internal friction
 * angle (c2 = cos^2 delta_int) and the basal friction t = tan delta_b:
 *   K_x = 2 (1 -/+ sqrt(1 - c2 (1 + t^2))) / c2 - 1,
 *   K_y = (K_x + 1 -/+ sqrt((K_x - 1)^2 + 4 t^2)) / 2,
 * the upper sign (active) where the flow extends in that direction, the lower
 * (passive) where it is compressed. */
static double ep_kx(double c2, double t, int active)
{
    double disc = 1.0 - c2 * (1.0 + t * t);
    double r = sqrt(disc > 0.0 ? disc : 0.0);
    return 2.0 * (active ? 1.0 - r : 1.0 + r) / c2 - 1.0;
}

static double ep_ky(double kx, double t, int active)
{
    double r = sqrt((kx - 1.0) * (kx - 1.0) + 4.0 * t * t);
    return 0.5 * (active ? kx + 1.0 - r : kx + 1.0 + r);
}

/* reading: the largest coefficient a cell can take (passive K_x, then the
 * passive K_y of it), bounding the solid's pressure speed in the CFL step
 * so that the time step needs no neighbour values. */
static double ep_kmax(double c2, double t) { return ep_ky(ep_kx(c2, t, 0), t, 0); }

/* reading: per cell, active in X where the central difference of the
 * (desingularised) solid velocity v_X^s along xi is >= 0, passive otherwise;
 * likewise in Y with v_Y^s along eta; from the extended stage input.  A ghost
 * cell takes the coefficients of the cell its boundary rule maps it to. */
static void earth_pressure(ora_sim *o)
{
    size_t np = (size_t)o->px * o->py;
    const double *m = o->Ue, *px = o->Ue + np, *py = o->Ue + 2 * np;
    for (int j = 0; j < o->ny; j++)
        for (int i = 0; i < o->nx; i++) {
            size_t e = PIDX(o, i + 1, j), w = PIDX(o, i - 1, j), n = PIDX(o, i, j + 1), s = PIDX(o, i, j - 1);
            double dvx = desing(px[e], m[e], o->md) - desing(px[w], m[w], o->md);
            double dvy = desing(py[n], m[n], o->md) - desing(py[s], m[s], o->md);
            double t = o->tan_mu ? o->tan_mu[CIDX(o, i, j)] : o->tan_d;
            double kx = ep_kx(o->cos2_int, t, dvx >= 0.0);
            o->Kx[PIDX(o, i, j)] = kx;
            o->Ky[PIDX(o, i, j)] = ep_ky(kx, t, dvy >= 0.0);
        }
    for (int j = -HALO; j < o->ny + HALO; j++)
        for (int i = -HALO; i < o->nx + HALO; i++) {
            if (i >= 0 && i < o->nx && j >= 0 && j < o->ny) continue;
            int f = 0;
            int ii = map_index(i, o->nx, o->p.bc[0], o->p.bc[1], &f);
            int jj = map_index(j, o->ny, o->p.bc[2], o->p.bc[3], &f);
            o->Kx[PIDX(o, i, j)] = o->Kx[PIDX(o, ii, jj)];
            o->Ky[PIDX(o, i, j)] = o->Ky[PIDX(o, ii, jj)];
        }
}

/* ------------------------------------------------------- inflow (Mode II) */

static double interp(const double *t, const double *y, int n, double tau)
{
    if (tau <= t[0]) return y[0];
    if (tau >= t[n - 1]) return y[n - 1];
    int k = 0;
    while (k + 1 < n && t[k + 1] < tau) k++;
    double w = (tau - t[k]) / (t[k + 1] - t[k]);
    return y[k] + w * (y[k + 1] - y[k]);
}

/* Cube root of x > 0 rounded to the double whose cube lies nearest to x:
 * from the library's cbrt(x) (a few units in the last place off, and
 * differently so on other platforms) step to the neighbour with the smaller
 * exact residual |y^3 - x| until neither neighbour is smaller (the residual
 * is unimodal in y, so every start ends on the same double).  It is formed with
 * error-free products (y^2 = p + e, y p = q + f exactly by fused
 * multiply-add; q - x is exact because q and x are within a factor of two),
 * which leaves only the tiny y e term rounded. */
static double cube_residual(double y, double x)
{
    double p = y * y;
    double e = fma(y, y, -p);
    double q = y * p;
    double f = fma(y, p, -q);
    double g = y * e;
    return ((q - x) + f) + g;
}

static double cbrt_nearest(double x)
{
    double y = cbrt(x);
    if (!(x > 0.0) || !isfinite(x)) return y;
    double r = fabs(cube_residual(y, x));
    for (int it = 0; it < 16; it++) {
        double lo = nextafter(y, 0.0), hi = nextafter(y, INFINITY);
        double rl = fabs(cube_residual(lo, x)), rh = fabs(cube_residual(hi, x));
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

/* reading: the inflow segment imposes the boundary face flux.  The discharge
 * per unit width q = Q / (ncells * face length) enters as a critical-depth
 * state (Froude number 1 over a flat bed): m_in = (q^2 / eps)^(1/3),
 * v_in = q / m_in, split into the phases by the hydrograph solid fraction. */
static void inflow_state(const ora_sim *o, const inflow_seg *s, double tau_nd,
                         double *q, double *m_in, double *v_in, double *phi)
{
    double tau = tau_nd * o->T;
    double Q = interp(s->t, s->Q, s->nt, tau);
    double ph = interp(s->t, s->phi, s->nt, tau);
    double w = (s->side < 2) ? o->p.dy : o->p.dx;
    double qs = Q / ((double)s->ncells * w);    /* m^2/s */
    double qn = qs / (o->p.H * o->V);            /* dimensionless */
    double m = cbrt_nearest(qn * qn / o->eps);
    *q = qn;
    *m_in = m;
    *v_in = m > 0.0 ? qn / m : 0.0;
    *phi = ph;
}

/* --------------------------------------------------------------- fluxes */

/* Physical flux of one reconstructed side of a face, from the flux vectors
 * F^s, G^s, F^f, G^f of Appendix A with the owner cell's geometry.
 * d = 0: xi direction (F), d = 1: eta direction (G).  Returns the flux, the
 * conserved values used by the numerical diffusion (momenta recomputed from
 * the desingularised velocities) and the local speeds of the two phases. */
static void side_flux(const ora_sim *o, const double u[NF], const geo_t *g, int d,
                      double F[NF], double qv[NF], double a[2], double kep)
{
    double eps = o->eps, al = o->alpha;
    double ms = u[0], mf = u[3];
    double hs = ms / g->J, hf = mf / g->J, h = hs + hf;
    double vXs = desing(u[1], ms, o->md), vYs = desing(u[2], ms, o->md);
    double vXf = desing(u[4], mf, o->md), vYf = desing(u[5], mf, o->md);
    /* depth-averaged solid pressure, times the earth-pressure coefficient kep
     * of the flux direction (1 in the paper's model) */
    double Ns = kep * (g->c * (1.0 - al) * hs / 2.0);
    double pf = g->c * h / 2.0;               /* mean fluid pressure */
    double Ax = d == 0 ? g->A11 : g->A21;     /* weight of the X-momentum pressure term */
    double Ay = d == 0 ? g->A12 : g->A22;     /* weight of the Y-momentum pressure term */
    double Ann = d == 0 ? g->A11 : g->A22;
    double vns = d == 0 ? vXs : vYs;          /* v_xi = v_X, v_eta = v_Y (reading) */
    double vnf = d == 0 ? vXf : vYf;
    /* solid */
    F[0] = ms * vns;
    F[1] = ms * vXs * vns + eps * g->J * h * Ax * Ns;
    F[2] = ms * vYs * vns + eps * g->J * h * Ay * Ns;
    /* fluid */
    F[3] = mf * vnf;
    F[4] = mf * vXf * vnf + eps * g->J * h * Ax * pf;
    F[5] = mf * vYf * vnf + eps * g->J * h * Ay * pf;
    qv[0] = ms; qv[1] = ms * vXs; qv[2] = ms * vYs;
    qv[3] = mf; qv[4] = mf * vXf; qv[5] = mf * vYf;
    /* reading: phase speeds from the pressure terms, |v_n| + sqrt(dP/dm) */
    double cs = kep * (eps * Ann * g->c * (1.0 - al) * (h + hs) / 2.0);
    double cf = eps * Ann * g->c * h;
    a[0] = fabs(vns) + sqrt(cs > 0.0 ? cs : 0.0);
    a[1] = fabs(vnf) + sqrt(cf > 0.0 ? cf : 0.0);
}

/* One-sided speeds of one side of a face, per phase: the smallest and the
 * largest characteristic speed v_n -/+ sqrt(dP/dm) in the face normal
 * direction, from the same quantities as the speeds of side_flux. */
static void side_speeds(const ora_sim *o, const double u[NF], const geo_t *g, int d, double lo[2],
                        double hi[2], double kep)
{
    double eps = o->eps, al = o->alpha;
    double ms = u[0], mf = u[3];
    double hs = ms / g->J, hf = mf / g->J, h = hs + hf;
    double vns = desing(d == 0 ? u[1] : u[2], ms, o->md);
    double vnf = desing(d == 0 ? u[4] : u[5], mf, o->md);
    double Ann = d == 0 ? g->A11 : g->A22;
    double cs = kep * (eps * Ann * g->c * (1.0 - al) * (h + hs) / 2.0);
    double cf = eps * Ann * g->c * h;
    double rs = sqrt(cs > 0.0 ? cs : 0.0), rf = sqrt(cf > 0.0 ? cf : 0.0);
    lo[0] = vns - rs;
    hi[0] = vns + rs;
    lo[1] = vnf - rf;
    hi[1] = vnf + rf;
}

/* Central numerical flux at one face, per phase.
 * Default (Kurganov-Tadmor): H = (F(U-) + F(U+))/2 - a/2 (U+ - U-), a = max of
 * the phase's own speed on the two sides.
 * flags bit 2, central-upwind (the one-sided-speed form of the same central
 * scheme family, Kurganov-Noelle-Petrova, which Kurganov-Petrova 2007 builds
 * on): a+ = max(largest speed of the two sides, 0), a- = min(smallest speed of
 * the two sides, 0),
 *   H = (a+ F(U-) - a- F(U+)) / (a+ - a-) + a+ a- / (a+ - a-) (U+ - U-),
 * and (F(U-) + F(U+))/2 where a+ = a- = 0.  With a- = -a+ it is the
 * Kurganov-Tadmor flux. */
static void central_flux(const ora_sim *o, const double uL[NF], const geo_t *gL,
                         const double uR[NF], const geo_t *gR, int d, double H[NF], double kL, double kR,
                         const double *dqm)
{
    double FL[NF], FR[NF], qL[NF], qR[NF], aL[2], aR[2];
    side_flux(o, uL, gL, d, FL, qL, aL, kL);
    side_flux(o, uR, gR, d, FR, qR, aR, kR);
    /* jump of each conserved field across the face in the numerical
     * diffusion (the well-balanced option gives the masses' from eta) */
    double dq[NF];
    for (int k = 0; k < NF; k++) dq[k] = qR[k] - qL[k];
    if (dqm) {
        dq[0] = dqm[0];
        dq[3] = dqm[1];
    }
    if (o->p.flags & 4) {
        double loL[2], hiL[2], loR[2], hiR[2];
        side_speeds(o, uL, gL, d, loL, hiL, kL);
        side_speeds(o, uR, gR, d, loR, hiR, kR);
        for (int ph = 0; ph < 2; ph++) {
            double ap = hiL[ph] > hiR[ph] ? hiL[ph] : hiR[ph];
            double am = loL[ph] < loR[ph] ? loL[ph] : loR[ph];
            if (ap < 0.0) ap = 0.0;
            if (am > 0.0) am = 0.0;
            double den = ap - am;
            for (int k = 3 * ph; k < 3 * ph + 3; k++)
                H[k] = den > 0.0 ? (ap * FL[k] - am * FR[k]) / den + ap * am / den * dq[k]
                                 : 0.5 * (FL[k] + FR[k]);
        }
        return;
    }
    for (int ph = 0; ph < 2; ph++) {
        double a = aL[ph] > aR[ph] ? aL[ph] : aR[ph];
        for (int k = 3 * ph; k < 3 * ph + 3; k++)
            H[k] = 0.5 * (FL[k] + FR[k]) - 0.5 * a * dq[k];
    }
}

/* Prescribed flux of an inflow face.  ``sgn`` = +1 for W/S (inward +X/+Y),
 * -1 for E/N. */
static void inflow_flux(const ora_sim *o, const geo_t *g, int d, int sgn, double q, double m_in,
                        double v_in, double phi, double H[NF])
{
    double eps = o->eps, al = o->alpha;
    double h = m_in / g->J, hs = phi * m_in / g->J;
    double Ns = g->c * (1.0 - al) * hs / 2.0, pf = g->c * h / 2.0;
    double Ax = d == 0 ? g->A11 : g->A21, Ay = d == 0 ? g->A12 : g->A22;
    double qs = phi * q, qf = (1.0 - phi) * q;
    H[0] = sgn * qs;
    H[3] = sgn * qf;
    H[1] = eps * g->J * h * Ax * Ns + (d == 0 ? qs * v_in : 0.0);
    H[2] = eps * g->J * h * Ay * Ns + (d == 1 ? qs * v_in : 0.0);
    H[4] = eps * g->J * h * Ax * pf + (d == 0 ? qf * v_in : 0.0);
    H[5] = eps * g->J * h * Ay * pf + (d == 1 ? qf * v_in : 0.0);
}

static const inflow_seg *inflow_at(const ora_sim *o, int side, int k)
{
    for (int s = 0; s < o->nseg; s++)
        if (o->seg[s].side == side && k >= o->seg[s].i0 && k < o->seg[s].i0 + o->seg[s].ncells)
            return &o->seg[s];
    return NULL;
}

/* Face values by minmod-limited linear reconstruction of the conserved
 * fields (Sect. 2.2), at face (i+1/2, j) (d = 0) or (i, j+1/2) (d = 1). */
static void face_values(const ora_sim *o, int i, int j, int d, double uL[NF], double uR[NF])
{
    size_t np = (size_t)o->px * o->py;
    int di = d == 0 ? 1 : 0, dj = d == 0 ? 0 : 1;
    for (int k = 0; k < NF; k++) {
        const double *f = o->Ue + k * np;
        double wm = f[PIDX(o, i - di, j - dj)], w0 = f[PIDX(o, i, j)];
        double w1 = f[PIDX(o, i + di, j + dj)], w2 = f[PIDX(o, i + 2 * di, j + 2 * dj)];
        double s0 = minmod(w0 - wm, w1 - w0);
        double s1 = minmod(w1 - w0, w2 - w1);
        uL[k] = w0 + 0.5 * s0;
        uR[k] = w1 - 0.5 * s1;
    }
}

/* ---------------------------------- well-balanced option (flags bit 5)
 * reading (the well-balanced central-upwind line of work Sect. 2.2 cites,
 * with the hydrostatic reconstruction of Audusse et al. 2004 in this model's
 * variables): at rest (v = 0, kappa = 0) a phase's pressure flux through a
 * xi-face is (1 + b_Y^2) eta^2 / (2 eps) (times 1 - alpha for the solid) and
 * its basal-pressure source is -(eta / eps) b_X, with eta = eps c^2 m
 * (= eps c h); so on beds that vary in one direction, and on planes (where the
 * eta-faces' cross term closes it), the model's rest states are b + eta =
 * const per phase; on a general two-dimensional bed the two momentum
 * balances give two conditions for one thickness and the model has no rest
 * state besides the dry bed.  Per cell and direction: face
 * values of eta and of the bed by minmod; at a face, B* = max of the two bed
 * values, eta* = max(0, eta + b - B*) per side; the face flux from the starred
 * states (m* = eta* / (eps c^2), momenta m* times the side's velocity, the
 * masses' numerical diffusion on eta* with the larger 1 / (eps c^2) of the two
 * sides); each cell adds the difference of the
 * pressure terms of its own face state and the starred one; the hydrostatic
 * part of the basal-pressure source uses the mean of the cell's two face
 * values of eta and the difference of its two bed face values. */

static double hr_c2(const ora_sim *o, int ii, int jj, int d)
{
    int p = d == 0 ? ii : jj, n = d == 0 ? o->nx : o->ny;
    int st = p < -1 ? 1 : (p > n ? -1 : 0);
    int di = d == 0 ? st : 0, dj = d == 0 ? 0 : st;
    double c = o->G[PIDX(o, ii + di, jj + dj)].c;
    return c * c;
}

/* cell (i, j) along d: face values of eta of phase ph (em at i - 1/2, ep at
 * i + 1/2) and of the bed (bm, bp) */
static void hr_cell(const ora_sim *o, int i, int j, int d, int ph, double *em, double *ep, double *bm, double *bp)
{
    size_t np = (size_t)o->px * o->py;
    int di = d == 0 ? 1 : 0, dj = d == 0 ? 0 : 1;
    const double *f = o->Ue + (size_t)(3 * ph) * np;
    double eta[3], b[3];
    for (int q = 0; q < 3; q++) {
        int ii = i + (q - 1) * di, jj = j + (q - 1) * dj;
        eta[q] = o->eps * hr_c2(o, ii, jj, d) * f[PIDX(o, ii, jj)];
        b[q] = o->b[PIDX(o, ii, jj)];
    }
    double se = minmod(eta[1] - eta[0], eta[2] - eta[1]);
    double sb = minmod(b[1] - b[0], b[2] - b[1]);
    *em = eta[1] - 0.5 * se;
    *ep = eta[1] + 0.5 * se;
    *bm = b[1] - 0.5 * sb;
    *bp = b[1] + 0.5 * sb;
}

/* pressure parts of the side flux F (momentum components), the terms of side_flux */
static void hr_pterm(const ora_sim *o, const double u[NF], const geo_t *g, int d, double P[NF])
{
    double eps = o->eps, al = o->alpha;
    double hs = u[0] / g->J, hf = u[3] / g->J, h = hs + hf;
    double Ns = g->c * (1.0 - al) * hs / 2.0, pf = g->c * h / 2.0;
    double Ax = d == 0 ? g->A11 : g->A21, Ay = d == 0 ? g->A12 : g->A22;
    for (int k = 0; k < NF; k++) P[k] = 0.0;
    P[1] = eps * g->J * h * Ax * Ns;
    P[2] = eps * g->J * h * Ay * Ns;
    P[4] = eps * g->J * h * Ax * pf;
    P[5] = eps * g->J * h * Ay * pf;
}

/* 1 if a state-inflow segment covers boundary index k of a side */
static int hr_segment_at(const ora_sim *o, int side, int k)
{
    for (int s = 0; s < o->nsseg; s++)
        if (o->sseg[s].side == side && k >= o->sseg[s].i0 && k < o->sseg[s].i0 + o->sseg[s].ncells) return 1;
    return 0;
}

/* Well-balanced face (i, j) + 1/2 along d: starred states, flux H and the
 * corrections cL, cR of the left and right cell. */
static void hr_face(ora_sim *o, int i, int j, int d, const double uL[NF], const double uR[NF], double H[NF],
                    double cL[NF], double cR[NF])
{
    int di = d == 0 ? 1 : 0, dj = d == 0 ? 0 : 1;
    const geo_t *gL = &o->G[PIDX(o, i, j)], *gR = &o->G[PIDX(o, i + di, j + dj)];
    double c2L = hr_c2(o, i, j, d), c2R = hr_c2(o, i + di, j + dj, d);
    /* a wall face: the ghost side mirrors the edge cell (its face values of
     * eta and the bed, its c and geometry), so no mass crosses the wall and a
     * lake at rest stays at rest against it; not where a state-inflow segment
     * holds the ghost cells */
    int p = d == 0 ? i : j, n = d == 0 ? o->nx : o->ny, kb = d == 0 ? j : i;
    int wallL = p == -1 && o->p.bc[2 * d] == 1 && !hr_segment_at(o, 2 * d, kb);
    int wallR = p + 1 == n && o->p.bc[2 * d + 1] == 1 && !hr_segment_at(o, 2 * d + 1, kb);
    if (wallL) {
        gL = gR;
        c2L = c2R;
    }
    if (wallR) {
        gR = gL;
        c2R = c2L;
    }
    double sL[NF], sR[NF], dqm[2];
    for (int ph = 0; ph < 2; ph++) {
        double em, ep, bm, bp, fm, fp, gm, gp;
        hr_cell(o, i, j, d, ph, &em, &ep, &bm, &bp);
        hr_cell(o, i + di, j + dj, d, ph, &fm, &fp, &gm, &gp);
        double etaL = ep, bL = bp, etaR = fm, bR = gm;
        if (wallL) {
            etaL = etaR;
            bL = bR;
        }
        if (wallR) {
            etaR = etaL;
            bR = bL;
        }
        double Bs = bL > bR ? bL : bR;
        double esL = etaL + bL - Bs, esR = etaR + bR - Bs;
        if (esL < 0.0) esL = 0.0;
        if (esR < 0.0) esR = 0.0;
        int k0 = 3 * ph;
        double mL = etaL / (o->eps * c2L), mR = etaR / (o->eps * c2R);
        double msL = esL / (o->eps * c2L), msR = esR / (o->eps * c2R);
        /* starred face states: the masses from eta*, the momenta of the plain
         * reconstruction scaled by the same factor (the velocity is kept) */
        double fL = mL > 0.0 ? msL / mL : 0.0, fR = mR > 0.0 ? msR / mR : 0.0;
        sL[k0] = msL; sL[k0 + 1] = uL[k0 + 1] * fL; sL[k0 + 2] = uL[k0 + 2] * fL;
        sR[k0] = msR; sR[k0 + 1] = uR[k0 + 1] * fR; sR[k0 + 2] = uR[k0 + 2] * fR;
        /* mass diffusion weight: the larger 1 / (eps c^2) of the two sides,
         * so each side's diffusion covers its own flux m* v (no mass leaves a
         * dry cell next to a wet one on a different slope) */
        dqm[ph] = (esR - esL) * ((c2L < c2R ? 1.0 / c2L : 1.0 / c2R) / o->eps);
        /* unstarred face states for the pressure corrections */
        cL[k0] = mL; cL[k0 + 1] = uL[k0 + 1]; cL[k0 + 2] = uL[k0 + 2];
        cR[k0] = mR; cR[k0 + 1] = uR[k0 + 1]; cR[k0 + 2] = uR[k0 + 2];
    }
    central_flux(o, sL, gL, sR, gR, d, H, 1.0, 1.0, dqm);
    double PL[NF], PLs[NF], PR[NF], PRs[NF];
    hr_pterm(o, cL, gL, d, PL);
    hr_pterm(o, sL, gL, d, PLs);
    hr_pterm(o, cR, gR, d, PR);
    hr_pterm(o, sR, gR, d, PRs);
    for (int k = 0; k < NF; k++) {
        cL[k] = PL[k] - PLs[k];
        cR[k] = PR[k] - PRs[k];
    }
}

static void compute_fluxes(ora_sim *o, double tau)
{
    int nx = o->nx, ny = o->ny;
    size_t nfx = (size_t)(nx + 1) * ny, nfy = (size_t)nx * (ny + 1);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++)
        for (int i = -1; i < nx; i++) {
            double uL[NF], uR[NF], H[NF];
            face_values(o, i, j, 0, uL, uR);
            size_t f = (size_t)j * (nx + 1) + (size_t)(i + 1);
            if (o->p.flags & 32) {
                double cL[NF], cR[NF];
                hr_face(o, i, j, 0, uL, uR, H, cL, cR);
                for (int k = 0; k < NF; k++) {
                    o->HXcL[k * nfx + f] = cL[k];
                    o->HXcR[k * nfx + f] = cR[k];
                }
            } else {
                const int ep = (o->p.flags & 8) != 0;
                central_flux(o, uL, &o->G[PIDX(o, i, j)], uR, &o->G[PIDX(o, i + 1, j)], 0, H,
                             ep ? o->Kx[PIDX(o, i, j)] : 1.0, ep ? o->Kx[PIDX(o, i + 1, j)] : 1.0, NULL);
            }
            for (int k = 0; k < NF; k++) o->HX[k * nfx + f] = H[k];
        }
#pragma omp parallel for schedule(static)
    for (int j = -1; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            double uL[NF], uR[NF], H[NF];
            face_values(o, i, j, 1, uL, uR);
            size_t f = (size_t)(j + 1) * nx + (size_t)i;
            if (o->p.flags & 32) {
                double cL[NF], cR[NF];
                hr_face(o, i, j, 1, uL, uR, H, cL, cR);
                for (int k = 0; k < NF; k++) {
                    o->HYcL[k * nfy + f] = cL[k];
                    o->HYcR[k * nfy + f] = cR[k];
                }
            } else {
                const int ep = (o->p.flags & 8) != 0;
                central_flux(o, uL, &o->G[PIDX(o, i, j)], uR, &o->G[PIDX(o, i, j + 1)], 1, H,
                             ep ? o->Ky[PIDX(o, i, j)] : 1.0, ep ? o->Ky[PIDX(o, i, j + 1)] : 1.0, NULL);
            }
            for (int k = 0; k < NF; k++) o->HY[k * nfy + f] = H[k];
        }
    /* Mode-II: prescribed fluxes on the inflow faces */
    for (int s = 0; s < o->nseg; s++) {
        const inflow_seg *sg = &o->seg[s];
        double q, m_in, v_in, phi;
        inflow_state(o, sg, tau, &q, &m_in, &v_in, &phi);
        for (int k = sg->i0; k < sg->i0 + sg->ncells; k++) {
            double H[NF];
            size_t f;
            if (sg->side == 0) { /* W: face -1/2 of cell (0, k) */
                inflow_flux(o, &o->G[PIDX(o, 0, k)], 0, +1, q, m_in, v_in, phi, H);
                f = (size_t)k * (nx + 1);
                for (int c = 0; c < NF; c++) o->HX[c * nfx + f] = H[c];
            } else if (sg->side == 1) { /* E: face nx-1/2 of cell (nx-1, k) */
                inflow_flux(o, &o->G[PIDX(o, nx - 1, k)], 0, -1, q, m_in, v_in, phi, H);
                f = (size_t)k * (nx + 1) + (size_t)nx;
                for (int c = 0; c < NF; c++) o->HX[c * nfx + f] = H[c];
            } else if (sg->side == 2) { /* S: face -1/2 of cell (k, 0) */
                inflow_flux(o, &o->G[PIDX(o, k, 0)], 1, +1, q, m_in, v_in, phi, H);
                f = (size_t)k;
                for (int c = 0; c < NF; c++) o->HY[c * nfy + f] = H[c];
            } else { /* N */
                inflow_flux(o, &o->G[PIDX(o, k, ny - 1)], 1, -1, q, m_in, v_in, phi, H);
                f = (size_t)ny * nx + (size_t)k;
                for (int c = 0; c < NF; c++) o->HY[c * nfy + f] = H[c];
            }
        }
    }
}

/* Net outward mass flux rate through the non-inflow boundary faces. */
static void boundary_outflow(const ora_sim *o, double out[2])
{
    int nx = o->nx, ny = o->ny;
    size_t nfx = (size_t)(nx + 1) * ny, nfy = (size_t)nx * (ny + 1);
    out[0] = out[1] = 0.0;
    for (int ph = 0; ph < 2; ph++) {
        const double *hx = o->HX + (size_t)(3 * ph) * nfx, *hy = o->HY + (size_t)(3 * ph) * nfy;
        double acc = 0.0;
        for (int j = 0; j < ny; j++) {
            if (!inflow_at(o, 0, j)) acc -= hx[(size_t)j * (nx + 1)] * o->deta;
            if (!inflow_at(o, 1, j)) acc += hx[(size_t)j * (nx + 1) + nx] * o->deta;
        }
        for (int i = 0; i < nx; i++) {
            if (!inflow_at(o, 2, i)) acc -= hy[i] * o->dxi;
            if (!inflow_at(o, 3, i)) acc += hy[(size_t)ny * nx + i] * o->dxi;
        }
        out[ph] = acc;
    }
}

static double inflow_rate(const ora_sim *o, double tau, int ph)
{
    double acc = 0.0;
    for (int s = 0; s < o->nseg; s++) {
        double q, m_in, v_in, phi;
        inflow_state(o, &o->seg[s], tau, &q, &m_in, &v_in, &phi);
        double w = (o->seg[s].side < 2) ? o->deta : o->dxi;
        acc += (ph == 0 ? phi * q : (1.0 - phi) * q) * (double)o->seg[s].ncells * w;
    }
    return acc;
}

/* -------------------------------------------------------------- sources */

typedef struct {
    double kappa[2];
    double sn[2][2], sf[2][2], sv[2][2], sd[2], svis[2], phis, phif;
} src_t;

static double fluid_G(const ora_sim *o, int i, int j)
{
    /* J_b h pbar^f with pbar^f = c h / 2 (Appendix A) */
    size_t np = (size_t)o->px * o->py, q = PIDX(o, i, j);
    const geo_t *g = &o->G[q];
    double h = (o->Ue[0 * np + q] + o->Ue[3 * np + q]) / g->J;
    return g->J * h * (g->c * h / 2.0);
}

static void fluid_vel(const ora_sim *o, int i, int j, double *u, double *w)
{
    size_t np = (size_t)o->px * o->py, q = PIDX(o, i, j);
    *u = desing(o->Ue[4 * np + q], o->Ue[3 * np + q], o->md);
    *w = desing(o->Ue[5 * np + q], o->Ue[3 * np + q], o->md);
}

static double mix_Jh(const ora_sim *o, int i, int j)
{
    size_t np = (size_t)o->px * o->py, q = PIDX(o, i, j);
    return o->Ue[0 * np + q] + o->Ue[3 * np + q]; /* J_b h */
}

/* Viscous term s_vis^f (Appendix A) in conservative face form.
 * reading: at a face the normal derivative is the neighbour difference, the
 * tangential derivative the mean of the two adjacent central differences,
 * J_b h and A_ij the arithmetic means of the two cells. */
static void viscous(const ora_sim *o, int i, int j, double S[2])
{
    double FX[2], FY[2], GX[2], GY[2];
    for (int side = 0; side < 2; side++) {
        /* x-face between (ia, j) and (ia+1, j) */
        int ia = side == 0 ? i - 1 : i;
        double u0, w0, u1, w1;
        fluid_vel(o, ia, j, &u0, &w0);
        fluid_vel(o, ia + 1, j, &u1, &w1);
        double un0, wn0, us0, ws0, un1, wn1, us1, ws1;
        fluid_vel(o, ia, j + 1, &un0, &wn0);
        fluid_vel(o, ia, j - 1, &us0, &ws0);
        fluid_vel(o, ia + 1, j + 1, &un1, &wn1);
        fluid_vel(o, ia + 1, j - 1, &us1, &ws1);
        double dxu = (u1 - u0) / o->dxi, dxw = (w1 - w0) / o->dxi;
        double dyu = 0.5 * ((un0 - us0) / (2.0 * o->deta) + (un1 - us1) / (2.0 * o->deta));
        double dyw = 0.5 * ((wn0 - ws0) / (2.0 * o->deta) + (wn1 - ws1) / (2.0 * o->deta));
        const geo_t *ga = &o->G[PIDX(o, ia, j)], *gb = &o->G[PIDX(o, ia + 1, j)];
        double Jh = 0.5 * (mix_Jh(o, ia, j) + mix_Jh(o, ia + 1, j));
        double A11 = 0.5 * (ga->A11 + gb->A11), A12 = 0.5 * (ga->A12 + gb->A12);
        double A21 = 0.5 * (ga->A21 + gb->A21), A22 = 0.5 * (ga->A22 + gb->A22);
        FX[side] = 2.0 * Jh * (A11 * dxu + A21 * dyu);
        FY[side] = Jh * (A12 * dxu + A22 * dyu + A11 * dxw + A21 * dyw);
    }
    for (int side = 0; side < 2; side++) {
        /* y-face between (i, ja) and (i, ja+1) */
        int ja = side == 0 ? j - 1 : j;
        double u0, w0, u1, w1;
        fluid_vel(o, i, ja, &u0, &w0);
        fluid_vel(o, i, ja + 1, &u1, &w1);
        double ue0, we0, uw0, ww0, ue1, we1, uw1, ww1;
        fluid_vel(o, i + 1, ja, &ue0, &we0);
        fluid_vel(o, i - 1, ja, &uw0, &ww0);
        fluid_vel(o, i + 1, ja + 1, &ue1, &we1);
        fluid_vel(o, i - 1, ja + 1, &uw1, &ww1);
        double dyu = (u1 - u0) / o->deta, dyw = (w1 - w0) / o->deta;
        double dxu = 0.5 * ((ue0 - uw0) / (2.0 * o->dxi) + (ue1 - uw1) / (2.0 * o->dxi));
        double dxw = 0.5 * ((we0 - ww0) / (2.0 * o->dxi) + (we1 - ww1) / (2.0 * o->dxi));
        const geo_t *ga = &o->G[PIDX(o, i, ja)], *gb = &o->G[PIDX(o, i, ja + 1)];
        double Jh = 0.5 * (mix_Jh(o, i, ja) + mix_Jh(o, i, ja + 1));
        double A11 = 0.5 * (ga->A11 + gb->A11), A12 = 0.5 * (ga->A12 + gb->A12);
        double A21 = 0.5 * (ga->A21 + gb->A21), A22 = 0.5 * (ga->A22 + gb->A22);
        GX[side] = Jh * (A12 * dxu + A22 * dyu + A11 * dxw + A21 * dyw);
        GY[side] = 2.0 * Jh * (A12 * dxw + A22 * dyw);
    }
    S[0] = (FX[1] - FX[0]) / o->dxi + (GX[1] - GX[0]) / o->deta;
    S[1] = (FY[1] - FY[0]) / o->dxi + (GY[1] - GY[0]) / o->deta;
}

/* All source terms at interior cell (i, j) from the stage-input state
 * (Appendix A, momentum balances of the solid and the fluid). */
static void sources(const ora_sim *o, int i, int j, src_t *S)
{
    size_t np = (size_t)o->px * o->py, q = PIDX(o, i, j), c = CIDX(o, i, j);
    const geo_t *g = &o->G[q];
    double eps = o->eps, al = o->alpha;
    double ms = o->Ue[0 * np + q], mf = o->Ue[3 * np + q];
    double hs = ms / g->J, hf = mf / g->J, h = hs + hf;
    double mt = ms + mf;
    /* volume fractions phi = h^{s,f} / h, desingularised like the velocities */
    double phis = desing(ms, mt, o->md), phif = desing(mf, mt, o->md);
    double v[2][3];
    v[0][0] = desing(o->Ue[1 * np + q], ms, o->md);
    v[0][1] = desing(o->Ue[2 * np + q], ms, o->md);
    v[1][0] = desing(o->Ue[4 * np + q], mf, o->md);
    v[1][1] = desing(o->Ue[5 * np + q], mf, o->md);
    for (int ph = 0; ph < 2; ph++) /* tangency: v_Z = b_X v_X + b_Y v_Y */
        v[ph][2] = g->bX * v[ph][0] + g->bY * v[ph][1];
    const double *dx = o->dnx + 3 * c, *dy = o->dny + 3 * c;
    for (int ph = 0; ph < 2; ph++) {
        /* centripetal acceleration: sum_k v_k (dn_k/dxi v_xi + dn_k/deta v_eta) */
        double k = 0.0;
        for (int a = 0; a < 3; a++) k += v[ph][a] * dx[a] * v[ph][0];
        for (int a = 0; a < 3; a++) k += v[ph][a] * dy[a] * v[ph][1];
        S->kappa[ph] = k;
    }
    /* basal pressures; reading: clamped at zero (no tensile basal contact) */
    double pbs = hs * (g->c * (1.0 - al) - o->eps_chi * S->kappa[0]);
    double pbf = hf * (g->c - o->eps_chi * S->kappa[1]);
    if (pbs < 0.0) pbs = 0.0;
    if (pbf < 0.0) pbf = 0.0;
    S->sn[0][0] = g->J * pbs * g->nX; S->sn[0][1] = g->J * pbs * g->nY;
    S->sn[1][0] = g->J * pbf * g->nX; S->sn[1][1] = g->J * pbf * g->nY;
    if (o->p.flags & 32) {
        /* well-balanced option: the hydrostatic part J h c n of s_n (with
         * (1 - alpha) for the solid) in the form that balances the face
         * corrections: -(fac / eps) (mean face eta) (bed face difference) / step */
        for (int ph = 0; ph < 2; ph++) {
            double fac = ph == 0 ? 1.0 - al : 1.0;
            double hph = ph == 0 ? hs : hf;
            double pb = ph == 0 ? pbs : pbf;
            if (!(pb > 0.0)) continue; /* lifted off: no normal force */
            for (int d = 0; d < 2; d++) {
                double em, ep, bm, bp;
                hr_cell(o, i, j, d, ph, &em, &ep, &bm, &bp);
                double nd = d == 0 ? g->nX : g->nY;
                double hydro = g->J * hph * g->c * fac * nd;
                double wb = -(fac / eps) * (0.5 * (em + ep)) * (bp - bm) / (d == 0 ? o->dxi : o->deta);
                S->sn[ph][d] += wb - hydro;
            }
        }
    }
    /* interphase pressure: gradient of J_b h pbar^f by central differences */
    double dGx = (fluid_G(o, i + 1, j) - fluid_G(o, i - 1, j)) / (2.0 * o->dxi);
    double dGy = (fluid_G(o, i, j + 1) - fluid_G(o, i, j - 1)) / (2.0 * o->deta);
    double gx = g->A11 * dGx + g->A21 * dGy;
    double gy = g->A12 * dGx + g->A22 * dGy;
    S->sf[0][0] = -eps * al * phis * gx;
    S->sf[0][1] = -eps * al * phis * gy;
    /* reading: the fluid term is weighted by phi^s (printed phi^f cancels the
     * fluid's own pressure gradient in the pure-fluid limit) */
    double wf = (o->p.flags & 1) ? phif : phis;
    S->sf[1][0] = eps * wf * gx;
    S->sf[1][1] = eps * wf * gy;
    /* interphase drag */
    double Kd = g->J * o->p.c_d * phis * phif * h;
    S->sv[0][0] = al * Kd * (v[1][0] - v[0][0]);
    S->sv[0][1] = al * Kd * (v[1][1] - v[0][1]);
    S->sv[1][0] = -Kd * (v[1][0] - v[0][0]);
    S->sv[1][1] = -Kd * (v[1][1] - v[0][1]);
    /* fluid basal friction */
    double fr = g->J * phif * h * o->p.theta_b * o->p.inv_n_r / eps;
    S->sd[0] = -fr * v[1][0];
    S->sd[1] = -fr * v[1][1];
    /* fluid viscosity */
    if (o->p.inv_n_r != 0.0) {
        double Sv[2];
        viscous(o, i, j, Sv);
        S->svis[0] = eps * phif * o->p.inv_n_r * Sv[0];
        S->svis[1] = eps * phif * o->p.inv_n_r * Sv[1];
    } else {
        S->svis[0] = S->svis[1] = 0.0;
    }
    S->phis = phis;
    S->phif = phif;
}

/* ----------------------------------------------------------------- stage */

/* One forward-Euler stage E(U) at stage time tau with step dt. */
static void stage(ora_sim *o, const double *Uin, double *Uout, double dt, double tau, int st)
{
    int nx = o->nx, ny = o->ny;
    size_t nc = (size_t)nx * ny, nfx = (size_t)(nx + 1) * ny, nfy = (size_t)nx * (ny + 1);
    size_t np = (size_t)o->px * o->py;
    extend_state(o, Uin, tau);
    if (o->p.flags & 8) earth_pressure(o);
    compute_fluxes(o, tau);
    boundary_outflow(o, o->bflux[st]);
    int64_t clamps = 0;
#pragma omp parallel for schedule(static) reduction(+ : clamps)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            size_t c = CIDX(o, i, j), q = PIDX(o, i, j);
            const geo_t *g = &o->G[q];
            src_t S;
            sources(o, i, j, &S);
            double out[NF];
            for (int k = 0; k < NF; k++) {
                double dFx = o->HX[k * nfx + (size_t)j * (nx + 1) + i + 1] - o->HX[k * nfx + (size_t)j * (nx + 1) + i];
                double dGy = o->HY[k * nfy + (size_t)(j + 1) * nx + i] - o->HY[k * nfy + (size_t)j * nx + i];
                if (o->p.flags & 32) {
                    dFx += o->HXcL[k * nfx + (size_t)j * (nx + 1) + i + 1] - o->HXcR[k * nfx + (size_t)j * (nx + 1) + i];
                    dGy += o->HYcL[k * nfy + (size_t)(j + 1) * nx + i] - o->HYcR[k * nfy + (size_t)j * nx + i];
                }
                double r = -dFx / o->dxi - dGy / o->deta;
                int ph = k / 3, comp = k % 3;
                if (comp > 0) {
                    int a = comp - 1;
                    r += S.sn[ph][a];
                    r += S.sf[ph][a];
                    r += S.sv[ph][a];
                    if (ph == 1) {
                        r += S.sd[a];
                        r += S.svis[a];
                    }
                }
                out[k] = o->Ue[k * np + q] + dt * r;
            }
            /* Coulomb basal friction of the solid, -J p_b tan(delta) v/|v|, as a
             * stop-clamp.  reading: the impulse F = dt J p_b tan(delta) removes
             * momentum along the tentative 3-D direction and stops the grains
             * when |q_3D| <= F (|q_3D| includes v_Z = b_X v_X + b_Y v_Y).  The
             * basal pressure is taken with the tentative solid thickness (the
             * centripetal term from the stage input), so that grains entering a
             * cell that was empty at the stage start feel friction at once. */
            double tmu = o->tan_mu ? o->tan_mu[c] : o->tan_d;
            double hst = out[0] / g->J;
            double pbt = hst * (g->c * (1.0 - o->alpha) - o->eps_chi * S.kappa[0]);
            if (pbt < 0.0) pbt = 0.0;
            double F = dt * (g->J * pbt) * tmu;
            double pX = out[1], pY = out[2];
            double pZ = g->bX * pX + g->bY * pY;
            if (o->p.flags & 16) {
                /* smooth friction, for finite-difference checks of gradients
                 * (the stop-clamp has a kink at rest): the Coulomb term
                 * -F v / sqrt(|v|^2 + v_eps^2) in a form that never reverses
                 * the flow, p = p~ r / (r + F) with
                 * r = sqrt(|p~_3D|^2 + (m~^s v_eps)^2), smooth in p~ and F */
                if (F > 0.0) {
                    double me = out[0] * (o->p.v_eps / o->V);
                    double r = sqrt(pX * pX + pY * pY + pZ * pZ + me * me);
                    out[1] = pX * (r / (r + F));
                    out[2] = pY * (r / (r + F));
                }
            } else {
                double p3 = sqrt(pX * pX + pY * pY + pZ * pZ);
                if (p3 <= F) {
                    out[1] = 0.0;
                    out[2] = 0.0;
                } else {
                    out[1] = pX * (1.0 - F / p3);
                    out[2] = pY * (1.0 - F / p3);
                }
            }
            /* positivity; reading: a phase without mass carries no momentum */
            for (int ph = 0; ph < 2; ph++)
                if (out[3 * ph] <= 0.0) {
                    if (out[3 * ph] < 0.0) clamps++;
                    out[3 * ph] = 0.0;
                    out[3 * ph + 1] = 0.0;
                    out[3 * ph + 2] = 0.0;
                }
            for (int k = 0; k < NF; k++) Uout[k * nc + c] = out[k];
        }
    o->clamps += clamps;
}

/* ------------------------------------------------------------------- dt */

/* Largest local speeds over all cells and phases (Sect. 2.2, Sect. 3.1.2:
 * the global maximum wave speed), plus inflow and floor. */
static void max_speeds(const ora_sim *o, double amax[2])
{
    size_t nc = (size_t)o->nx * o->ny;
    double ax = 0.0, ay = 0.0;
    for (int j = 0; j < o->ny; j++)
        for (int i = 0; i < o->nx; i++) {
            size_t c = CIDX(o, i, j);
            double u[NF], F[NF], qv[NF], a[2];
            for (int k = 0; k < NF; k++) u[k] = o->U[k * nc + c];
            const geo_t *g = &o->G[PIDX(o, i, j)];
            double km = 1.0;
            if (o->p.flags & 8) km = ep_kmax(o->cos2_int, o->tan_mu ? o->tan_mu[c] : o->tan_d);
            side_flux(o, u, g, 0, F, qv, a, km);
            if (a[0] > ax) ax = a[0];
            if (a[1] > ax) ax = a[1];
            side_flux(o, u, g, 1, F, qv, a, km);
            if (a[0] > ay) ay = a[0];
            if (a[1] > ay) ay = a[1];
        }
    for (int s = 0; s < o->nseg; s++) {
        double q, m_in, v_in, phi;
        inflow_state(o, &o->seg[s], o->t, &q, &m_in, &v_in, &phi);
        double a = v_in + sqrt(o->eps * m_in);
        if (o->seg[s].side < 2) { if (a > ax) ax = a; }
        else if (a > ay) ay = a;
    }
    /* reading: a state-inflow ghost moves at most |v| + sqrt(eps m) */
    for (int s = 0; s < o->nsseg; s++) {
        double u[NF], m, v;
        ghost_state(o, &o->sseg[s], o->t, u, &m, &v);
        double a = fabs(v) + sqrt(o->eps * m);
        if (o->sseg[s].side < 2) { if (a > ax) ax = a; }
        else if (a > ay) ay = a;
    }
    double fl = o->p.a_min / o->V;
    amax[0] = ax > fl ? ax : fl;
    amax[1] = ay > fl ? ay : fl;
}

static double next_dt(const ora_sim *o, double t_end_nd)
{
    double a[2];
    max_speeds(o, a);
    double dtx = o->dxi / a[0], dty = o->deta / a[1];
    double dt = o->p.cfl * (dtx < dty ? dtx : dty);
    if (o->n_sched > 0 && o->steps < o->n_sched) dt = o->dt_sched[o->steps]; /* frozen steps */
    if (t_end_nd - o->t < dt) dt = t_end_nd - o->t;
    if (dt < 0.0) dt = 0.0;
    return dt;
}

/* ----------------------------------------------------------------- step */

/* One step of the two-step modified Euler method (Heun / SSP-RK2, the
 * paper's choice, Sect. 2.2): U* = E(U^n), U** = E(U*),
 * U^{n+1} = (U^n + U**) / 2.  With flags bit 1, the three-stage SSP
 * Runge-Kutta method of the same family (the "multi-step RK" the paper
 * names as an option): U1 = E(U^n), U2 = 3/4 U^n + 1/4 E(U1),
 * U^{n+1} = 1/3 U^n + 2/3 E(U2), stage times t, t + dt, t + dt/2 and
 * quadrature weights 1/6, 1/6, 2/3 for the boundary integrals.  Returns dt
 * in s. */
double ora_step(ora_sim *o, double t_end_si)
{
    size_t nc = (size_t)o->nx * o->ny;
    double t_end = t_end_si / o->T;
    double dt = next_dt(o, t_end);
    if (dt <= 0.0) return 0.0;
    const int rk3 = (o->p.flags & 2) != 0;
    stage(o, o->U, o->Us, dt, o->t, 0);
    stage(o, o->Us, o->Uss, dt, o->t + dt, 1);
    if (rk3) {
        for (size_t k = 0; k < NF * nc; k++) o->Us[k] = 0.75 * o->U[k] + 0.25 * o->Uss[k];
        stage(o, o->Us, o->Uss, dt, o->t + 0.5 * dt, 2);
        for (size_t k = 0; k < NF * nc; k++) o->U[k] = (1.0 / 3.0) * o->U[k] + (2.0 / 3.0) * o->Uss[k];
    } else {
        for (size_t k = 0; k < NF * nc; k++) o->U[k] = 0.5 * (o->U[k] + o->Uss[k]);
    }
    double scale = o->p.H * o->p.L * o->p.L; /* dimensionless volume -> m^3 */
    for (int ph = 0; ph < 2; ph++) {
        double out, in;
        if (rk3) {
            out = dt * (o->bflux[0][ph] / 6.0 + o->bflux[1][ph] / 6.0 + 2.0 * o->bflux[2][ph] / 3.0);
            in = dt * (inflow_rate(o, o->t, ph) / 6.0 + inflow_rate(o, o->t + dt, ph) / 6.0 +
                       2.0 * inflow_rate(o, o->t + 0.5 * dt, ph) / 3.0);
        } else {
            out = 0.5 * dt * (o->bflux[0][ph] + o->bflux[1][ph]);
            in = 0.5 * dt * (inflow_rate(o, o->t, ph) + inflow_rate(o, o->t + dt, ph));
        }
        if (ph == 0) { o->out_s += out * scale; o->in_s += in * scale; }
        else { o->out_f += out * scale; o->in_f += in * scale; }
    }
    o->t += dt;
    o->steps++;
    o->last_dt = dt * o->T;
    return dt * o->T;
}

/* Prescribe the time steps (s) of steps 0 .. n-1 (n = 0 clears). */
void ora_set_dt_schedule(ora_sim *o, const double *dts, int64_t n)
{
    free(o->dt_sched);
    o->dt_sched = NULL;
    o->n_sched = 0;
    if (n <= 0) return;
    o->dt_sched = (double *)xcalloc((size_t)n, sizeof(double));
    for (int64_t k = 0; k < n; k++) o->dt_sched[k] = dts[k] / o->T;
    o->n_sched = n;
}

/* Run ``nsteps`` steps (or until t_end); dt history (s) into dt_hist if given. */
int64_t ora_run(ora_sim *o, int64_t nsteps, double t_end_si, double *dt_hist)
{
    int64_t n = 0;
    for (; n < nsteps; n++) {
        double dt = ora_step(o, t_end_si);
        if (dt <= 0.0) break;
        if (dt_hist) dt_hist[n] = dt;
    }
    return n;
}

/* Next step's dt (s) without stepping. */
double ora_peek_dt(const ora_sim *o, double t_end_si) { return next_dt(o, t_end_si / o->T) * o->T; }

/* Diagnostics: t (s), steps, volume of solid and fluid (m^3), inflow and
 * outflow volumes per phase (m^3), positivity clamps, last dt (s). */
void ora_diag(const ora_sim *o, double out[10])
{
    size_t nc = (size_t)o->nx * o->ny;
    double ms = 0.0, mf = 0.0;
    for (size_t c = 0; c < nc; c++) { ms += o->U[c]; mf += o->U[3 * nc + c]; }
    double scale = o->p.H * o->p.L * o->p.L * o->dxi * o->deta;
    out[0] = o->t * o->T;
    out[1] = (double)o->steps;
    out[2] = ms * scale;
    out[3] = mf * scale;
    out[4] = o->in_s; out[5] = o->in_f; out[6] = o->out_s; out[7] = o->out_f;
    out[8] = (double)o->clamps;
    out[9] = o->last_dt;
}

/* Output fields of the paper (Sect. 3.1.2, Stage 3): bed-normal thickness h
 * (m), solid fraction, horizontal velocities of both phases (m/s). */
void ora_get_fields(const ora_sim *o, double *h, double *phi_s, double *vxs, double *vys,
                    double *vxf, double *vyf)
{
    size_t nc = (size_t)o->nx * o->ny;
    for (int j = 0; j < o->ny; j++)
        for (int i = 0; i < o->nx; i++) {
            size_t c = CIDX(o, i, j);
            double J = o->G[PIDX(o, i, j)].J;
            double ms = o->U[c], mf = o->U[3 * nc + c], mt = ms + mf;
            if (h) h[c] = mt / J * o->p.H;
            if (phi_s) phi_s[c] = desing(ms, mt, o->md);
            if (vxs) vxs[c] = desing(o->U[1 * nc + c], ms, o->md) * o->V;
            if (vys) vys[c] = desing(o->U[2 * nc + c], ms, o->md) * o->V;
            if (vxf) vxf[c] = desing(o->U[4 * nc + c], mf, o->md) * o->V;
            if (vyf) vyf[c] = desing(o->U[5 * nc + c], mf, o->md) * o->V;
        }
}

/* Probe for tests: geometry and source terms at interior cell (i, j) for the
 * current state.  out[0..9]: bX, bY, J, c, nX, nY, nZ, A11, A12, A22;
 * out[10..15]: dn/dxi (3), dn/deta (3); out[16..17]: kappa^s, kappa^f;
 * out[18..33]: s_n, s_f, s_v (solid X,Y then fluid X,Y each), s_d^f, s_vis^f. */
void ora_probe(ora_sim *o, int i, int j, double out[34])
{
    extend_state(o, o->U, o->t);
    const geo_t *g = &o->G[PIDX(o, i, j)];
    size_t c = CIDX(o, i, j);
    out[0] = g->bX; out[1] = g->bY; out[2] = g->J; out[3] = g->c;
    out[4] = g->nX; out[5] = g->nY; out[6] = g->nZ;
    out[7] = g->A11; out[8] = g->A12; out[9] = g->A22;
    for (int a = 0; a < 3; a++) { out[10 + a] = o->dnx[3 * c + a]; out[13 + a] = o->dny[3 * c + a]; }
    src_t S;
    sources(o, i, j, &S);
    out[16] = S.kappa[0]; out[17] = S.kappa[1];
    int k = 18;
    for (int ph = 0; ph < 2; ph++) { out[k++] = S.sn[ph][0]; out[k++] = S.sn[ph][1]; }
    for (int ph = 0; ph < 2; ph++) { out[k++] = S.sf[ph][0]; out[k++] = S.sf[ph][1]; }
    for (int ph = 0; ph < 2; ph++) { out[k++] = S.sv[ph][0]; out[k++] = S.sv[ph][1]; }
    out[k++] = S.sd[0]; out[k++] = S.sd[1];
    out[k++] = S.svis[0]; out[k++] = S.svis[1];
}

/* Probe for tests: one forward-Euler stage E(U) of the scheme (Sect. 2.2) from
 * the current state at the current time with the step dt (s), written to
 * Uout (raw layout, 6 * nx * ny).  The state, time, counters and boundary
 * integrals are left as they were. */
void ora_stage_probe(ora_sim *o, double dt_si, double *Uout)
{
    int64_t clamps = o->clamps;
    double bf[3][2];
    memcpy(bf, o->bflux, sizeof bf);
    stage(o, o->U, Uout, dt_si / o->T, o->t, 0);
    o->clamps = clamps;
    memcpy(o->bflux, bf, sizeof bf);
}

/* Probe for tests: the cube root the critical depth uses. */
double ora_cbrt_nearest(double x) { return cbrt_nearest(x); }

/* Scales for tests: eps, alpha, T (s), V (m/s), dxi, deta, md. */
void ora_scales(const ora_sim *o, double out[7])
{
    out[0] = o->eps; out[1] = o->alpha; out[2] = o->T; out[3] = o->V;
    out[4] = o->dxi; out[5] = o->deta; out[6] = o->md;
}
