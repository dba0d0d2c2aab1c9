/*
 * m2p.h -- C ABI of the MI355X (gfx950) two-phase shallow-flow step.
 *
 * The library advances the depth-integrated grain-fluid model of MoSES_2PDF
 * (Ko, Chen, Wong, Tai; model equations in the paper's Appendix A, numerics in
 * Sect. 2.2) on a DEM grid: minmod-limited reconstruction, central
 * (Kurganov-Tadmor) fluxes, topography / Coulomb-friction / fluid-friction /
 * buoyancy / viscous / interphase-drag sources, Mode-I release and Mode-II
 * inflow boundaries (Sect. 3.1.2, Stage 0), the two-step modified Euler
 * (Heun) time integrator and a CFL-limited global time step (Sect. 2.2).
 *
 * Conventions shared by every entry point:
 *  - Every function returns int: 0 = M2P_OK, < 0 = an M2P_E* code.  No C++
 *    exception crosses the ABI.  m2p_last_error() gives a thread-local text.
 *  - Units at the ABI are SI (m, s, m/s, kg/m^3, degrees).  The library
 *    rescales internally (X, Y, b ~ L; h ~ H; v ~ sqrt(g L); t ~ sqrt(L/g)).
 *  - Host arrays are row-major [ny][nx] (y outer), cell-centred: cell (i, j)
 *    sits at X = (i + 1/2) dx, Y = (j + 1/2) dy.  They are copied at call
 *    time and never retained.
 *  - All device work is enqueued on the HIP stream given at creation (NULL =
 *    the default stream).  Calls that return host data synchronize that stream.
 *  - After a device-side error (non-finite value, dt floor) a context is
 *    poisoned: only m2p_get_*, m2p_get_diag and m2p_destroy are allowed.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef M2P_H
#define M2P_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define M2P_OK 0
#define M2P_EINVAL -1      /* bad sizes or values (phi outside [0,1], delta_b outside [0,90), cfl outside (0,1], non-finite DEM, ...) */
#define M2P_ENOMEM -2      /* device allocation failed */
#define M2P_EHIP -3        /* a HIP runtime call failed (text in m2p_last_error) */
#define M2P_ENONFINITE -4  /* the device saw a NaN or Inf in the state or in dt */
#define M2P_ENEGDEPTH -5   /* negative thickness handed to m2p_set_state or m2p_batch_set_state */
#define M2P_EDTFLOOR -6    /* the CFL time step fell below 1e-12 of the grid's gravity-wave time */
#define M2P_EMAXSTEPS -7   /* m2p_run_to stopped at max_steps before t_end */
#define M2P_ESTATE -8      /* call order (step before set_state, poisoned context, ...) */
#define M2P_EIO -9         /* a file could not be opened, read or written */

/* arithmetic of the state: FP64, or FP32 state with FP64 time, dt and volume sums */
#define M2P_FP64 0
#define M2P_FP32 1

/* boundary mode per side (Sect. 3.1.2: the paper's default is non-reflecting) */
#define M2P_BC_TRANSMISSIVE 0 /* zero-gradient copy of the edge cell */
#define M2P_BC_WALL 1         /* mirror, normal momentum of both phases negated */

/* sides, in the order of m2p_params.bc */
#define M2P_SIDE_W 0
#define M2P_SIDE_E 1
#define M2P_SIDE_S 2
#define M2P_SIDE_N 3

/* m2p_params.flags */
#define M2P_F_FLUID_PRESSURE_AS_PRINTED 1 /* weight the fluid interphase pressure by phi^f as printed */
#define M2P_F_RK3 2 /* three-stage third-order SSP Runge-Kutta instead of the paper's two-step modified Euler
                       (Heun): U1 = E(U^n), U2 = 3/4 U^n + 1/4 E(U1), U^{n+1} = 1/3 U^n + 2/3 E(U2) at stage
                       times t, t + dt, t + dt/2 (Sect. 2.2 names multi-step Runge-Kutta methods as the family);
                       single-scenario contexts only, not with the adjoint */
#define M2P_F_CENTRAL_UPWIND 4 /* central-upwind face flux with one-sided local speeds instead of the Kurganov-Tadmor
                       central flux: per phase a+ = max(largest characteristic speed v_n + sqrt(dP/dm) of the two
                       sides, 0), a- = min(smallest speed v_n - sqrt(dP/dm), 0), H = (a+ F- - a- F+) / (a+ - a-)
                       + a+ a- / (a+ - a-) (U+ - U-), (F- + F+) / 2 on a dry face (Sect. 2.2 builds on the central
                       schemes of Kurganov-Tadmor 2000 and Kurganov-Petrova 2007; this is the latter's flux without
                       its well-balanced surface reconstruction); single-scenario contexts only, not with the
                       tangent and adjoint calls */
#define M2P_F_EARTH_PRESSURE 8 /* Savage-Hutter earth-pressure coefficients on the solid pressure (the paper's model has
                       none, Appendix A): per cell and direction, active where the solid velocity's central
                       difference along the direction is >= 0, else passive, K_x = 2 (1 -/+ sqrt(1 - cos^2 d_int
                       (1 + tan^2 d_b))) / cos^2 d_int - 1, K_y = (K_x + 1 -/+ sqrt((K_x - 1)^2 + 4 tan^2 d_b)) / 2,
                       d_int = delta_int_deg; needs delta_b (and every tan_mu) <= delta_int < 90 deg; Mode-I
                       releases on single-scenario contexts (the tiled kernel computes the coefficients in its
                       march; with M2P_F_CENTRAL_UPWIND the reference kernel runs the option after a coefficient
                       pass); not with the tangent and adjoint calls */

#define M2P_F_SMOOTH_FRICTION 16 /* smooth Coulomb friction, for finite-difference checks of gradients (the
                       stop-clamp of the paper's friction term has a kink at rest): after the tentative
                       update the solid momentum is scaled by r / (r + F), F = dt J_b p_b tan(delta_b) the
                       Coulomb impulse and r = sqrt(|p_3D|^2 + (m^s v_eps)^2), a regularised form of
                       -F v / sqrt(|v|^2 + v_eps^2) that never reverses the flow; a layer below the
                       friction angle creeps instead of resting.  Needs v_eps > 0; single-scenario
                       contexts, run by the reference kernel; differentiated by the tangent and adjoint */
#define M2P_F_WELL_BALANCED 32 /* well-balanced hydrostatic reconstruction of the face states (Sect. 2.2 cites the
                       well-balanced central-upwind schemes; this is the reconstruction of Audusse et al. 2004 in
                       the model's variables): per phase eta = eps c^2 m; per cell and direction minmod face values
                       of eta and of the bed; at a face B* = max of the two bed values, eta* = max(0, eta + b - B*)
                       per side, the flux from the starred states (m* = eta* / (eps c^2), momenta scaled by m* / m,
                       the masses' numerical diffusion on eta* weighted with the larger 1 / (eps c^2) of the two
                       sides, which keeps dry cells positive), each cell adding the pressure terms of its
                       unstarred minus its starred face state; the hydrostatic part of the basal-pressure source
                       becomes -(fac / eps) (mean face eta) (bed face difference) / step (fac = 1 - alpha for the
                       solid, 1 for the fluid).  A wall face mirrors the edge cell.  Keeps a lake at rest on beds
                       that vary in one direction and the model's other states to the scheme's order;
                       single-scenario contexts, both kernel variants (the tiled kernel has its own instance,
                       FP64 results bitwise equal to the reference kernel's; with state-inflow segments the
                       reference kernel runs); with either face flux; Mode-II inflow only as state segments
                       (m2p_set_inflow_states; a wall face that a segment covers is not mirrored): m2p_set_inflow
                       returns M2P_EINVAL for discharge segments; not with M2P_F_EARTH_PRESSURE, ensembles, the
                       tangent and adjoint calls (m2p_create returns M2P_EINVAL for the combination) */

/* thickness convention of m2p_set_state */
#define M2P_DEPTH_NORMAL 0   /* h measured normal to the bed (the paper's h, Sect. 2.1) */
#define M2P_DEPTH_VERTICAL 1 /* vertical thickness */

/* kernel variants (m2p_set_variant) */
#define M2P_VARIANT_AUTO 0
#define M2P_VARIANT_REFERENCE 1 /* one thread per cell, every stencil value from memory */
#define M2P_VARIANT_TILED 2     /* fused LDS-free column-marching stage kernel */
#define M2P_VARIANT_TILED_GLOBAL 3 /* the tiled kernel with 64-bit global addresses instead of raw buffer
                                      accesses, as used where the state or the DEM exceeds 2 GiB */

typedef struct m2p_ctx m2p_ctx;

typedef struct {
    int32_t nx, ny; /* cells; both >= 4 */
    double dx, dy;  /* cell size (m) */
} m2p_grid;

/* Material and numerical parameters (Sect. 3.1.2, Stage 1; Table 1). */
typedef struct {
    double delta_b_deg;   /* basal friction angle delta_b, [0, 90) */
    double c_d;           /* interphase drag coefficient C_d */
    double inv_n_r;       /* 1 / N_R; 0 switches fluid friction and viscosity off */
    double theta_b;       /* fluid basal friction coefficient */
    double rho_s, rho_f;  /* densities; alpha_rho = rho_f / rho_s */
    double delta_int_deg; /* internal friction angle: used by M2P_F_EARTH_PRESSURE only */
    double cfl;           /* CFL number, (0, 1]; the paper uses 0.1 */
    double L, H;          /* length and thickness scales (m); aspect ratio eps = H / L */
    double chi;           /* exponent of eps on the centripetal term of the basal pressure */
    double g;             /* gravity (m/s^2) */
    double m_dry;         /* desingularisation thickness (m) for velocities and fractions */
    double a_min;         /* floor of the CFL wave speed (m/s) */
    int32_t bc[4];        /* M2P_BC_* for W, E, S, N */
    int32_t flags;        /* M2P_F_* */
    double v_eps;         /* regularisation speed (m/s) of M2P_F_SMOOTH_FRICTION (> 0 with it; else unused) */
} m2p_params;

/* One Mode-II inflow segment (Sect. 3.1.2, Stage 0; Sect. 4.2): ncells
 * boundary cells from index i0 along ``side`` receive a prescribed face flux
 * from a piecewise-linear hydrograph of discharge Q (m^3/s) and solid
 * fraction over time t (s), nt >= 1 samples, t increasing. */
typedef struct {
    int32_t side, i0, ncells, nt;
    const double *t, *Q, *phi_s;
} m2p_inflow;

/* Mode-II inflow segment given as the state of the inflowing flow (the
 * paper's inflow condition: hydrographs of flow thickness, solid fraction and
 * velocity at boundary locations, Sect. 3.1.2 Stage 0): ncells boundary cells
 * from i0 on side; piecewise-linear hydrographs over time t (s, increasing,
 * nt >= 1 samples) of the vertical flow thickness h (m, >= 0), the solid
 * fraction phi_s and the speed v (m/s) of both phases along the inward
 * boundary normal.  The two ghost cells outside each segment cell hold this
 * state at the stage time and the boundary face flux is the scheme's central
 * flux; the flow through these faces enters the out_s / out_f integrals of
 * m2p_diag (negative for inflow). */
typedef struct {
    int32_t side, i0, ncells, nt;
    const double *t, *h, *phi_s, *v;
} m2p_inflow_state;

typedef struct {
    double t;            /* model time (s) */
    double dt_last;      /* last step (s) */
    double dt_next;      /* step the next m2p_step will take (s) */
    double mass_s, mass_f; /* volume of each phase (m^3), FP64 sums */
    double in_s, in_f;   /* inflow volumes accumulated (m^3) */
    double out_s, out_f; /* outflow volumes accumulated through non-inflow boundary faces (m^3) */
    int64_t steps;       /* steps taken */
    int64_t clamp_count; /* positivity clamps (tentative negative thickness) */
    int32_t status;      /* device status bits: 1 non-finite, 2 dt floor */
    int32_t pad;
} m2p_diag;

/* Version string. */
const char *m2p_version(void);

/* Text for a status code; thread-local detail of the last failure. */
const char *m2p_strerror(int code);
const char *m2p_last_error(void);

/* Number of visible HIP devices (0 when none), without creating a context. */
int m2p_device_count(int *count);

/* Create a context on the current HIP device: copies the DEM (metres, ny*nx,
 * host) and optionally a per-cell friction field tan_mu (tan(delta_b) per
 * cell, ny*nx, host; NULL = uniform delta_b).  prec is M2P_FP64 or M2P_FP32.
 * hip_stream is a hipStream_t (NULL = default stream).  The context owns all
 * device memory unless m2p_bind_buffers is used.  Errors: EINVAL, ENOMEM, EHIP. */
int m2p_create(m2p_ctx **out, const m2p_grid *g, const m2p_params *p, int32_t prec,
               const double *dem_host, const double *tan_mu_host, void *hip_stream);

/* Destroy; frees what the context owns (never caller-bound buffers). */
void m2p_destroy(m2p_ctx *c);

/* Bytes of each of the two state buffers (6 fields, row pitch rounded up to
 * 64 elements) for a grid and precision. */
int m2p_buffer_bytes(const m2p_grid *g, int32_t prec, size_t *state_bytes);

/* Optional: use caller-owned device buffers (for example torch tensors) as
 * the two state buffers, each at least m2p_buffer_bytes long and 256-byte
 * aligned.  Must precede m2p_set_state; the buffers must outlive the context. */
int m2p_bind_buffers(m2p_ctx *c, void *state_a, void *state_b, size_t bytes);

/* Mode-I release or any state from SI host fields (ny*nx each): thickness h
 * (depth_kind M2P_DEPTH_NORMAL or M2P_DEPTH_VERTICAL), solid fraction in
 * [0, 1], horizontal velocities of solid and fluid (NULL = 0).  Resets nothing
 * else (time, integrals and step count persist).  Errors: ENEGDEPTH (a finite
 * h < 0), EINVAL (non-finite values, solid fraction outside [0, 1]), EHIP. */
int m2p_set_state(m2p_ctx *c, int32_t depth_kind, const double *h, const double *phi_s,
                  const double *vxs, const double *vys, const double *vxf, const double *vyf);

/* Raw conserved state, dimensionless, host FP64 [6][ny][nx]:
 * (m^s, p^s_X, p^s_Y, m^f, p^f_X, p^f_Y) with m = J_b h (the paper's
 * J_b h^s, J_b h^f and the momenta q^s, q^f).  get synchronizes. */
int m2p_set_state_raw(m2p_ctx *c, const double *U);
int m2p_get_state_raw(m2p_ctx *c, double *U);

/* Model time (s). */
int m2p_set_time(m2p_ctx *c, double t);

/* Mode-II inflow segments (replaces earlier ones); at most 8; arrays copied. */
int m2p_set_inflow(m2p_ctx *c, const m2p_inflow *seg, int32_t nseg);

/* Replace the Mode-II state segments (m2p_inflow_state; 0..8; nseg = 0
 * clears).  Segments may not share a boundary cell with each other or with a
 * discharge segment.  Errors: M2P_EINVAL. */
int m2p_set_inflow_states(m2p_ctx *c, const m2p_inflow_state *seg, int32_t nseg);

/* Select the stage-kernel variant (M2P_VARIANT_*); results are identical in
 * FP64.  tile_rows: rows each wavefront of the tiled variant marches, 1..4096,
 * or 0 = chosen from the grid size.  Errors: M2P_EINVAL. */
int m2p_set_variant(m2p_ctx *c, int32_t variant, int32_t tile_rows);

/* Choose the tile height of the tiled variant by timing: run trial_steps
 * steps (1..10000) at each of a few heights around the size rule's on the
 * context itself, putting the state, time, integrals and step count back
 * after each trial, and keep the fastest (results do not depend on the
 * height in either precision).  Returns the height and its ms per step (may
 * be NULL).  Synchronizes.  Errors: EINVAL (reference variant selected),
 * ESTATE, ENOMEM, EHIP. */
int m2p_autotune(m2p_ctx *c, int32_t trial_steps, int32_t *rows, double *ms_per_step);

/* One time step, enqueued.  If dt_out is not NULL the stream is synchronized
 * and the step taken (s) is returned (0 once t reached the run_to end time). */
int m2p_step(m2p_ctx *c, double *dt_out);

/* Enqueue nsteps steps without any host synchronization. */
int m2p_run(m2p_ctx *c, int64_t nsteps);

/* Steps are replayed from a HIP graph of `chunk` steps (default 32; 0 =
 * launch kernel by kernel) when the context has a stream of its own and
 * per-kernel profiling is off; the graph is captured on first use and again
 * whenever the constants, buffers or launch shape change.  Replays give the
 * same results as direct launches.  Errors: M2P_EINVAL for chunk outside
 * [0, 4096]. */
int m2p_set_graph(m2p_ctx *c, int32_t chunk);

/* Advance until t >= t_end (the last step is shortened to land on t_end) or
 * max_steps steps, checking the device status between chunks.  Returns
 * M2P_EMAXSTEPS if t_end was not reached. */
int m2p_run_to(m2p_ctx *c, double t_end, int64_t max_steps, int64_t *steps_done);

/* Run through the output times t_out[0..n_out) (s, increasing; the step
 * before each lands on it, as m2p_run_to) and store the output fields of
 * Sect. 3.1.2 Stage 3 at each: fields (host) is [n_out][6][ny][nx] with
 * h (bed-normal, m), phi_s, vxs, vys, vxf, vyf (m/s).  Each snapshot is
 * extracted on the device and copied to pinned host memory on a second
 * stream while the next interval is computed (two slots, allocated on first
 * use and kept until m2p_destroy).  max_steps bounds the steps of the whole
 * call; steps_done (may be NULL) returns them.  Errors: EINVAL, ESTATE,
 * EMAXSTEPS (outputs before the stop are stored), device errors. */
int m2p_run_outputs(m2p_ctx *c, const double *t_out, int64_t n_out, int64_t max_steps, double *fields,
                    int64_t *steps_done);

/* Output fields of the paper (Sect. 3.1.2, Stage 3), SI, host, ny*nx each,
 * NULL skips: bed-normal thickness h, solid fraction, v_X, v_Y of the solid
 * and of the fluid.  Synchronizes. */
int m2p_get_fields(m2p_ctx *c, double *h, double *phi_s, double *vxs, double *vys, double *vxf,
                   double *vyf);

/* Diagnostics (FP64 volume sums computed on demand).  Synchronizes. */
int m2p_get_diag(m2p_ctx *c, m2p_diag *d);

/* Wait for all work of the context. */
int m2p_synchronize(m2p_ctx *c);

/* Per-kernel timing with HIP events recorded on the context's stream around
 * each kernel of every step while on != 0 (adds one event record per kernel). */
int m2p_set_profiling(m2p_ctx *c, int32_t on);

/* Synchronize, then return the summed durations (ms) of the stage-1, stage-2
 * and finalize kernels of the steps timed since the last call, and their
 * number; resets the sums. */
int m2p_kernel_times(m2p_ctx *c, double *ms3, int64_t *nsteps);

/* Device pointer of the current state buffer and its row pitch (elements);
 * field k starts at ptr + k * ny * pitch. */
int m2p_state_device_ptr(m2p_ctx *c, void **ptr, int64_t *pitch);

/* Floating-point work of one cell in one stage of the forward step (the
 * scheme of Sect. 2.2 on the model of Appendix A), for rooflines.  Counted on
 * the host by running one cell's share of the stage kernel's arithmetic --
 * its geometry, one x-face and one y-face central flux, one new neighbour
 * difference per direction and field, sources, viscous face terms, update
 * and clamps, and in stage 2 the Heun average and CFL speeds -- through the
 * kernels' own device functions with an operation-counting number type, on
 * a wet sliding cell (the longer branch of the Coulomb clamp).
 * stage: 1 or 2.  visc: nonzero when the viscous term is on (inv_n_r > 0).
 * out[5] (host): additions and subtractions, multiplications, divisions,
 * square roots, comparisons (min / max / sign tests).  FLOPs are the sum of
 * the first four.  M2P_EINVAL for another stage or NULL out.  Needs no GPU. */
int m2p_stage_flops(int32_t stage, int32_t visc, double *out);

/* ---------------------------------------------------------------------------
 * GIS raster input and output: the DEM and initial fields come from GIS
 * systems as ASCII grids and results go back in that form (Sect. 1;
 * Sect. 3.1.2, Stages 1 and 3).  ESRI ASCII grid: header keys ncols, nrows,
 * xllcorner|xllcenter, yllcorner|yllcenter, cellsize, optional NODATA_value
 * (case-insensitive), then nrows lines of ncols values, northernmost first.
 * Arrays here are row-major ny*nx with row 0 at the southern edge.
 * ------------------------------------------------------------------------- */

/* Read an ESRI ASCII grid.  Fills g (nx = ncols, ny = nrows, dx = dy =
 * cellsize), the lower-left cell corner (x0, y0; may be NULL) and the NODATA
 * value (NaN when the file has none; may be NULL).  values (host, capacity
 * doubles) may be NULL to read the header only; NODATA cells are returned as
 * NaN, so a grid with missing cells cannot reach m2p_create or m2p_set_state
 * unnoticed (both reject non-finite values): fill them explicitly first.  Errors: M2P_EIO (open), M2P_EINVAL (malformed header, too few or
 * too many values, capacity < nx*ny). */
int m2p_esri_read(const char *path, m2p_grid *g, double *x0, double *y0, double *nodata, double *values,
                  size_t capacity);

/* Write values (host, ny*nx, row 0 south) as an ESRI ASCII grid with the
 * lower-left corner (x0, y0); non-finite values are written as nodata.
 * Needs square cells (dx == dy).  Errors: M2P_EINVAL, M2P_EIO. */
int m2p_esri_write(const char *path, const m2p_grid *g, double x0, double y0, double nodata, const double *values);

/* ---------------------------------------------------------------------------
 * Gradients (back-calculation of friction and release volume, the paper's
 * motivation in Sect. 1 and Sect. 5).  The step is differentiated with the
 * time steps held fixed ("frozen dt"); non-smooth points (minmod, wave-speed
 * maximum, Coulomb stop, positivity) take the derivative of the branch the
 * values select.  Mode-I only.
 * ------------------------------------------------------------------------- */

/* Set (or replace) the per-cell friction field tan(delta_b), host ny*nx. */
int m2p_set_friction_field(m2p_ctx *c, const double *tan_mu);

/* Prescribe the time steps (s) of the next n steps counted from step 0 of the
 * context (n = 0 clears): step k uses dts[k] instead of the CFL step. */
int m2p_set_dt_schedule(m2p_ctx *c, const double *dts, int64_t n);

/* Loss 1/2 sum (h - h_target)^2 dx dy of the current state (h bed-normal, m;
 * target host ny*nx). */
int m2p_loss(m2p_ctx *c, const double *target_h, double *loss);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight calibration or serving loops, harnesses that forbid
 * hipMalloc: the loss of m2p_loss with nothing allocated and no host
 * synchronization.  target_dev: device FP64 [ny][nx] target bed-normal
 * thickness (m), caller-owned; loss_dev: device FP64 scalar that receives
 * 1/2 sum (h - h_target)^2 dx dy (the same bits as m2p_loss).  Enqueued on
 * the context's stream.  The kernels' 1024 per-block partial sums live in a
 * library-owned device array of 2048 doubles (16 KiB) on each GPU, held until
 * the process ends and shared by every call on that GPU: calls that overlap
 * on one GPU (other streams or threads) race.  Any grid size fits (the
 * partial count does not depend on it).  Errors: EINVAL (NULL argument),
 * ESTATE (no state), EHIP. */
int m2p_loss_noalloc(m2p_ctx *c, const double *target_dev, double *loss_dev);

/* One forward-Euler stage E at the current state with the next step's dt and
 * the inflow state of stage 0 or 1: E(U) and its directional derivative along
 * dU (and along dmu, the friction field, if not NULL); host [6][ny][nx] raw
 * state layout (m2p_get_state_raw), dmu ny*nx. */
int m2p_stage_jvp(m2p_ctx *c, int32_t stage, const double *dU, const double *dmu, double *E, double *dE);

/* Transpose of the same stage Jacobian applied to lam ([6][ny][nx]):
 * lam_in = (dE/dU)^T lam and gmu = (dE/dmu)^T lam (ny*nx, may be NULL). */
int m2p_stage_vjp(m2p_ctx *c, int32_t stage, const double *lam, double *lam_in, double *gmu);

/* From the current state (the release scaled by vol_scale), run nsteps steps
 * storing a checkpoint every ckpt_every steps and the time steps, evaluate the
 * loss against target_h, then sweep backwards segment by segment (recomputing
 * each segment's states) through the transposed stages.  With ckpt_every >=
 * nsteps the forward run writes the whole tape (U^n and U* of every step:
 * 2 nsteps state buffers of device memory) and nothing is recomputed; the
 * results are the same bits either way.  Returns the loss, dL/d(tan delta_b)
 * per cell (grad_mu, ny*nx, may be NULL) and dL/d(vol_scale) (may be NULL).
 * M2P_ENOMEM if the tape does not fit.  The context ends at the forward run's
 * final state. */
int m2p_adjoint_run(m2p_ctx *c, int64_t nsteps, int32_t ckpt_every, const double *target_h, double vol_scale,
                    double *loss, double *grad_mu, double *grad_vol);

/* ---------------------------------------------------------------------------
 * Batched ensembles: nscen independent scenarios of uneven size advanced
 * together (the paper's motivation of many runs for parameter back-calculation,
 * Sect. 1 and Sect. 5).  All states share one ragged SoA arena; one persistent
 * launch per RK stage walks a work list of (scenario, strip, row block) items;
 * every scenario keeps its own CFL step, time, integrals and status, so member
 * i advances exactly like a single-scenario context of the same tile height.
 * Step sequences are captured into a HIP graph and replayed.  Mode-I only (no
 * inflow segments).  Arrays are per scenario with that scenario's grid.
 * ------------------------------------------------------------------------- */
typedef struct m2p_batch m2p_batch;

/* grids, params, dems: nscen entries (1..2047); tan_mu NULL or nscen entries,
 * each NULL (uniform delta_b) or a per-cell tan(delta_b) field.  hip_stream
 * NULL = a private non-blocking stream.  Errors: EINVAL (any scenario), ENOMEM, EHIP. */
int m2p_batch_create(m2p_batch **out, int32_t nscen, const m2p_grid *grids, const m2p_params *params,
                     const double *const *dems, const double *const *tan_mu, int32_t prec, void *hip_stream);
void m2p_batch_destroy(m2p_batch *b);

/* State of scenario i from SI host fields, as m2p_set_state. */
int m2p_batch_set_state(m2p_batch *b, int32_t i, int32_t depth_kind, const double *h, const double *phi_s,
                        const double *vxs, const double *vys, const double *vxf, const double *vyf);

/* Enqueue nsteps steps of every scenario (graph-captured chunks, no host sync). */
int m2p_batch_run(m2p_batch *b, int64_t nsteps);

/* Wait; returns M2P_ENONFINITE / M2P_EDTFLOOR if any scenario's status is set. */
int m2p_batch_synchronize(m2p_batch *b);

/* Raw state, output fields and diagnostics of scenario i (as the single-context calls). */
int m2p_batch_get_state_raw(m2p_batch *b, int32_t i, double *U);
int m2p_batch_get_fields(m2p_batch *b, int32_t i, double *h, double *phi_s, double *vxs, double *vys,
                         double *vxf, double *vyf);
int m2p_batch_get_diag(m2p_batch *b, int32_t i, m2p_diag *d);

/* Tile rows per wavefront (>= 4) and persistent workgroups (0 = default). */
int m2p_batch_set_tile(m2p_batch *b, int32_t rows, int32_t blocks);

/* Steps per captured graph (0 = launch kernels directly). */
int m2p_batch_set_graph(m2p_batch *b, int32_t chunk);

/* Time trial_steps steps per candidate tile shape on the batch itself (state
 * and scalars restored after each trial) and keep the fastest. */
int m2p_batch_autotune(m2p_batch *b, int32_t trial_steps, int32_t *rows, int32_t *blocks, double *ms_per_step);

/* Scenario count, total cells, tile rows, persistent workgroups, work items. */
int m2p_batch_info(m2p_batch *b, int32_t *nscen, int64_t *cells, int32_t *rows, int32_t *blocks, int32_t *nwork);

#ifdef __cplusplus
}
#endif

#endif /* M2P_H */
