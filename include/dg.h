/*
 * dg.h -- C ABI of the MI355X discontinuous-Galerkin hydrodynamics library.
 *
 * The library evaluates the right-hand side of the DG weight equations of
 * Cernetic, Springel, Guillet & Pakmor (arXiv 2208.11131) for the compressible
 * Euler / Navier-Stokes equations on a uniform Cartesian mesh of cubic cells
 * with a per-cell Legendre basis (the tensor set Q_n or the total-degree set
 * P_n of Sec. 2.3), and advances them with SSP Runge-Kutta steps under a CFL
 * time step; with it come the positivity limiter (Sec. 4.2), the passive
 * tracer (Sec. 3.4) and the Ornstein-Uhlenbeck driving field (Sec. 7.1).
 *
 * Conventions shared by every call:
 *   - Order p (the `order` argument) = n + 1 = modes = Gauss points per axis,
 *     1 <= p <= 8 (Sec. 2.3, 2.4).  Modes per field: p^dim (tensor set Q_n)
 *     or p(p+1)/2, p(p+1)(p+2)/6 in 2D, 3D (total-degree set P_n).
 *   - State layout (device, float64, C-contiguous): w[cell][field][mode],
 *     cell = i + n0 (j + n1 k), mode = l_x + p (l_y + p l_z) (tensor basis;
 *     the total-degree basis of dg_options.basis = 1 stores its modes as
 *     stated there); fields
 *     (rho, rho v_x, rho v_y[, rho v_z], e[, c rho][, alpha]): dim + 2
 *     conserved fields, the passive tracer c rho when enabled (Sec. 3.4), and
 *     the artificial-viscosity field alpha when AV is enabled (Sec. 4.1).
 *     w_0 of each field is the cell mean (orthonormal basis, Sec. 2.2).
 *   - Every pointer argument named w, wdot, s_coeffs or R is a DEVICE pointer
 *     owned by the caller (e.g. a torch tensor), 8-byte aligned; w and wdot
 *     of dg_rhs / dg_step / dg_step_cfl / dg_max_dt / dg_batch_step must be 16-byte
 *     aligned (the state is moved in 16-byte groups; DG_EINVAL otherwise,
 *     torch and hipMalloc allocations are 256-byte aligned); `stream` is a
 *     hipStream_t passed as void* (NULL = default stream).  Calls enqueue work
 *     on that stream and return without waiting, except where stated.
 *   - Errors are reported by the return code; nothing aborts or throws across
 *     the ABI.  DG_EINVAL leaves every buffer untouched.
 *   - One context per stream at a time: calls on one context are not
 *     thread-safe and must not overlap on different streams.
 */
#ifndef DG_H
#define DG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_ctx dg_ctx;

typedef enum {
    DG_OK = 0,
    DG_EINVAL = -1,         /* invalid argument (no side effect) */
    DG_ENOMEM = -2,         /* device allocation failed */
    DG_EDEVICE = -3,        /* HIP runtime / launch error */
    DG_ENONPHYSICAL = -4,   /* a cell-mean density or pressure <= 0 (Sec. 4.2) */
    DG_ENONFINITE = -5,     /* a non-finite weight was produced */
    DG_EUNSUPPORTED = -6,   /* valid request this build does not implement */
    DG_ESCRATCH = -7        /* beyond the static scratch of dg_max_dt_noalloc */
} dg_status;

typedef enum { DG_BC_PERIODIC = 0, DG_BC_OUTFLOW = 1, DG_BC_WALL = 2 } dg_bc;

/* Mesh: dim in {2,3}; n[a] cells on [lo[a], hi[a]] along axis a (entries of
 * unused axes ignored).  Cells must be cubic: (hi-lo)/n equal on every axis
 * to 1e-12 relative (Sec. 2.1).  Non-periodic ends (the paper's problems are
 * periodic; these are this library's boundary readings) use a ghost cell
 * built from the boundary cell itself, on both ends of that axis:
 *   DG_BC_OUTFLOW  mirrored ghost w_ghost(l_a) = (-1)^{l_a} w(l_a)
 *                  (transmissive: the face states are equal).  At high
 *                  order it is not stable over many steps: a rounding-level
 *                  disturbance grows at the boundary (measured at p = 6 by
 *                  about 0.4 % per step);
 *   DG_BC_WALL     reflecting wall: the mirrored ghost with the momentum
 *                  component normal to the boundary negated (no mass flux
 *                  through the boundary; stable). */
typedef struct {
    int dim;
    int n[3];
    double lo[3], hi[3];
    int bc[3];
} dg_mesh;

/* Artificial viscosity (Sec. 4.1, eqs. timedependentviscosity and
 * viscosu_flux_with_factor): dalpha/dt = f_v max(0, -div v)
 *   + f_w max(0, dlnS/dt) [S > s_onset/p^2] - alpha p c_s / (f_tau h),
 * eps = scale * clamp(alpha, 0, alpha_max) * c_s * h / p.
 * Paper defaults: scale 1, f_v 2.5, f_tau 0.5, f_w 0.2, s_onset 1e-4,
 * alpha_max 1 (dg_av_defaults fills them). */
typedef struct {
    int enabled;
    double scale, f_v, f_tau, f_w, s_onset, alpha_max;
} dg_av_params;

/* Precision of the bulk arithmetic: FP64 everywhere, or FP32 for the
 * contractions, point fluxes, Riemann and recovery (state, RK combination,
 * time step and totals stay FP64). */
typedef enum { DG_PREC_FP64 = 0, DG_PREC_FP32_BULK = 1 } dg_precision;

/* Options (NULL = defaults): precision FP64; basis 0 = tensor set Q_n
 * (p^dim modes per field), 1 = total-degree set P_n of Sec. 2.3 (the modes
 * of degree l_x + l_y [+ l_z] <= n: (n+1)(n+2)/2 in 2D, (n+1)(n+2)(n+3)/6 in
 * 3D, stored in the order l_z, l_y, l_x ascending with l_x fastest; every
 * physics of the tensor basis; the interface recovery then uses the basis of
 * total degree <= n+1 and the sensor's top modes are those of total degree
 * n; not for batched ensembles); cfl =
 * f_CFL of eq. timestep (default 0.5);
 * launch tiles (0 = built-in tuned table): cells per volume block, faces per
 * face-kernel pencil, threads per volume / face block (multiples of 64,
 * at most 512).  Results do not depend on the tiles.  limiter = 1: the
 * positivity limiter of dg_limit acts on every state an RK stage writes
 * (default 0; not available for batched ensembles).  tracer = 1 adds the
 * passive tracer c rho (Sec. 3.4 eq. passivetracer) as a conserved field
 * after e: flux c rho v minus the diffusion eta rho grad c, eta =
 * tracer_eta >= 0 (default off; not with AV, not for batched ensembles). */
typedef struct {
    int precision;
    int basis;
    double cfl;
    int cells_per_block;
    int faces_per_block;
    int vol_threads;
    int face_threads;
    int limiter;
    int tracer;
    double tracer_eta;
} dg_options;

void dg_av_defaults(dg_av_params *av);
void dg_options_defaults(dg_options *opt);

/* Create a context: validates the mesh and physics, builds the basis,
 * quadrature and recovery tables (Sec. 2.3, 2.4, 3.2) and allocates the
 * library-owned device buffers (RK registers, face-flux buffer, sensor
 * scalars, time-step scalars).  gamma > 1; nu (kinematic viscosity) and
 * kappa (thermal diffusivity chi of Sec. 3.3) >= 0; av NULL or disabled =
 * no AV field.  Cell and face indices are 32-bit on the device: the product
 * over the axes of (n[a] + 1) must not exceed 2^31 - 1 (DG_EINVAL).  Uses
 * the current HIP device.  *out = NULL on error. */
dg_status dg_init(const dg_mesh *mesh, int order, double gamma, double nu, double kappa,
                  const dg_av_params *av, const dg_options *opt, dg_ctx **out);

/* Free the context and its device buffers (NULL is ignored). */
void dg_free(dg_ctx *ctx);

/* Number of doubles of a state array: cells * fields * dg_num_modes. */
size_t dg_state_len(const dg_ctx *ctx);
/* Number of fields per cell (dim + 2, + 1 with the tracer, + 1 with AV). */
int dg_num_fields(const dg_ctx *ctx);
/* Number of conserved fields (dim + 2, + 1 with the tracer): the values
 * dg_conserved_totals returns. */
int dg_num_conserved(const dg_ctx *ctx);
/* Stored modes per field: p^dim (Q_n) or the total-degree count (P_n). */
int dg_num_modes(const dg_ctx *ctx);

/* Shape of the context (host pointers, any may be NULL): dimension, order p,
 * number of cells and fields per cell.  A state array holds
 * ncells * nfields * dg_num_modes doubles, a forcing array (dg_set_forcing)
 * ncells * dim * dg_num_modes, a sensor-rate array ncells.  DG_EINVAL for
 * NULL ctx. */
dg_status dg_shape(const dg_ctx *ctx, int *dim, int *order, long long *ncells, int *nfields);

/* wdot = dw/dt of the weight equations (Sec. 2.2 eq. weight_evolution,
 * discretised as Sec. 2.4 eq. time_stepping_final_analytical_equation, with
 * the viscous and AV fluxes of Sec. 3 and 4).  w and wdot must not overlap.
 * The AV wiggle source uses the context's stored dlnS/dt of the previous
 * step (0 after dg_init). */
dg_status dg_rhs(dg_ctx *ctx, const double *w, double *wdot, void *stream);

/* One SSP Runge-Kutta step of size dt > 0, in place (Sec. 2.5): forward
 * Euler for p = 1, SSPRK(2,2) for p = 2, SSPRK(3,3) for p = 3, the 5-stage
 * 4th-order SSPRK(5,4) for p >= 4.  Stage 1 also stores dlnS/dt of w for the
 * next step's wiggle source.  Sets the context's device error flag when a
 * stage produces a non-positive cell-mean density/pressure or a non-finite
 * weight (read it with dg_check). */
dg_status dg_step(dg_ctx *ctx, double *w, double dt, void *stream);

/* As dg_step, with dt = f_CFL h / (2 p (c_max + v_max)) computed on the
 * device from w (eq. timestep) and never copied to the host; if dt_dev is
 * not NULL the step size (double) is also stored there (device pointer).
 *
 * HIP graphs: dg_rhs, dg_step, dg_step_cfl and dg_limit enqueue kernel
 * launches only (no allocation, copy, memset or synchronisation), so they
 * may be captured from `stream`.  A replay repeats the captured launches
 * with the captured pointers and scalars (dg_step's dt included).  With
 * artificial viscosity the context alternates two sensor-rate buffers from
 * step to step: capture an even number of steps.  A driving field that
 * dg_set_forcing left pending is evaluated by the next call, captured or
 * not; replays evaluate it again only if it was captured. */
dg_status dg_step_cfl(dg_ctx *ctx, double *w, double *dt_dev, void *stream);

/* Positivity limiter (Sec. 4.2) on w (device, in place), every cell: with
 * positive mean density rho_bar and mean pressure p_bar (from the cell-mean
 * conserved values), if the density at a limiter point (the volume Gauss
 * points and the Gauss points of the cell's faces) is below rho_bottom =
 * 1e-6 rho_bar, every weight of degree >= 1 of every field is multiplied by
 * (rho_bar - rho_bottom) / (rho_bar - rho_min); then those weights are halved
 * while the pressure at a limiter point is below 1e-6 p_bar (at most 60
 * times, then they are set to 0).  Cell means never change; cells with a
 * non-positive mean density or pressure are left alone.  With the `limiter`
 * option the steps apply it to every stage state; the initial state is the
 * caller's to limit (once, with this call).  FP64 in both precisions. */
dg_status dg_limit(dg_ctx *ctx, double *w, void *stream);

/* Time step of eq. timestep: maxima of the sound speed and of |v| over all
 * volume Gauss points of w.  Synchronises `stream`; *dt_out is a host
 * pointer.  cmax_out / vmax_out (host, may be NULL) receive the maxima. */
dg_status dg_max_dt(dg_ctx *ctx, const double *w, double *dt_out, double *cmax_out, double *vmax_out,
                    void *stream);

/* Allocation-free form of dg_max_dt, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Computes the same maxima and dt with the same kernels,
 * but the per-block partial maxima live in a static device array of the
 * library (64 KiB per device, taken at dg_init; at most 4096 partials, which
 * every mesh meets: a larger request returns DG_ESCRATCH) instead of the
 * context's buffer, and the result goes to a caller-owned DEVICE array out[3]
 * = {dt, c_max, v_max} (8-byte aligned) instead of the host.  Enqueues two
 * launches on `stream` and returns without waiting: no allocation, no copy,
 * no synchronisation.  The current device must be the context's.  Every call
 * on one device shares that device's array: calls that overlap in time on one
 * device (different streams, threads or contexts) race and must be ordered by
 * the caller. */
dg_status dg_max_dt_noalloc(dg_ctx *ctx, const double *w, double *out, void *stream);

/* Conserved totals sum_K |K| w_0 per conserved field (dg_num_conserved
 * values, host pointer `out`), deterministic compensated FP64 sums.  The integral of each
 * conserved density over the box (Sec. 2.1: w_0 is the cell mean of the
 * orthonormal expansion, so |K| w_0 is the cell's content); on periodic
 * boxes the scheme keeps these constant (Sec. 3, manifestly conservative
 * form with single-valued face fluxes).  Synchronises. */
dg_status dg_conserved_totals(dg_ctx *ctx, const double *w, double *out, void *stream);

/* Body-force acceleration field s (Sec. 7 driving): device array
 * [cell][dim][dg_num_modes] of DG coefficients (8-byte aligned), acting in
 * every later RHS as the momentum source rho s and energy source rho s.v,
 * projected on the basis.  The library evaluates s at the Gauss points into
 * its own device buffer (ncells * dim * order^dim values of the bulk type,
 * allocated by the first call; DG_ENOMEM if that fails).  It does so on the
 * stream of the next RHS evaluation, reading s_coeffs then: the caller keeps
 * the array alive and unchanged until that RHS, and calls dg_set_forcing
 * again after changing the coefficients.  NULL removes the forcing. */
dg_status dg_set_forcing(dg_ctx *ctx, const double *s_coeffs);

/* ---------------------------------------------------------------------------
 * Driving field (Sec. 7.1 Driving): s(x) = sum_k 2 Re(a_k exp(2 pi i k.x)) over
 * the integer wave vectors 1 <= |k|^2 <= k_max^2 (one of each pair +-k: the
 * one whose first non-zero component is positive; ordered by k_x, then k_y,
 * then k_z ascending; k_z = 0 in 2D), with complex amplitude vectors a_k that
 * follow an Ornstein-Uhlenbeck process (correlation time t_corr, stationary
 * standard deviation sigma0 |k|^(-5/3) per component, the k^(-5/3) scaling of
 * Sec. 7.1) and are kept solenoidal, a_k -= k (k.a_k) / |k|^2 (the Helmholtz
 * projection of Sec. 7.1).  The update runs on the host in FP64; the random
 * draws are the caller's.  The projection on the DG basis runs on the device
 * and produces the array dg_set_forcing takes.
 * ------------------------------------------------------------------------- */
typedef struct dg_forcing dg_forcing;

/* Driving field on the box of `mesh` (periodic unit-length box expected) for
 * order p and basis (0 tensor, 1 total degree: the layout of the projected
 * coefficients, as dg_options.basis); 1 <= kmax <= 4, t_corr > 0,
 * sigma0 >= 0.  Amplitudes start at 0.  Host allocation only (the device
 * table is allocated by the first dg_forcing_project).  *out = NULL on error. */
dg_status dg_forcing_init(const dg_mesh *mesh, int order, int basis, int kmax, double t_corr, double sigma0,
                          dg_forcing **out);
void dg_forcing_free(dg_forcing *f);
/* Number of modes (one per +-k pair), and their wave vectors (host int[nm][3]). */
int dg_forcing_num_modes(const dg_forcing *f);
dg_status dg_forcing_modes(const dg_forcing *f, int *kv);
/* Amplitudes, host double[nm][3][2] (re, im per component; the third
 * component unused in 2D). */
dg_status dg_forcing_get_amplitudes(const dg_forcing *f, double *amp);
dg_status dg_forcing_set_amplitudes(dg_forcing *f, const double *amp);
/* One OU step over dt > 0: every component becomes
 * e^{-dt/t_corr} a + sigma_k sqrt(1 - e^{-2 dt/t_corr}) (xi_re + i xi_im)/sqrt(2)
 * with the caller's standard normal draws noise[nm][3][2] (host), then the
 * solenoidal projection.  dt = +inf draws from the stationary law.  Host
 * only; non-finite draws are rejected (DG_EINVAL, amplitudes unchanged). */
dg_status dg_forcing_update(dg_forcing *f, const double *noise, double dt);
/* DG coefficients of s on every cell, s_coeffs (device, caller-owned,
 * [cell][dim][modes] doubles): (1/|K|) int_K s phi_l, each mode's cell
 * integral factorised into per-axis factors (1/2) int exp(i pi k_a h xi)
 * Pt_l(xi) dxi tabulated on the host (modes in the layout of the basis).
 * Copies the amplitudes to the device
 * (synchronising `stream`), then enqueues one kernel.  The device table is
 * the object's own: calls on one object must not overlap on different
 * streams. */
dg_status dg_forcing_project(dg_forcing *f, double *s_coeffs, void *stream);

/* Per-cell d ln S / dt used by the wiggle source (Sec. 4.1): copy from /
 * to a caller device array of ncells doubles (checkpointing, tests). */
dg_status dg_set_sensor_rate(dg_ctx *ctx, const double *R, void *stream);
dg_status dg_get_sensor_rate(dg_ctx *ctx, double *R, void *stream);

/* Synchronise `stream`, read and clear the device error flag: DG_OK,
 * DG_ENONPHYSICAL or DG_ENONFINITE. */
dg_status dg_check(dg_ctx *ctx, void *stream);

/* Launch tiles in use (cells per volume block, threads per volume block,
 * faces per face block, threads per face block). */
dg_status dg_get_tiles(const dg_ctx *ctx, int *vol_cells, int *vol_threads, int *face_cells,
                       int *face_threads);

/* Kernel timing (instrumentation): when enabled, every face, volume and CFL
 * kernel launch of this context (the limiter counts as a CFL-kind launch)
 * is bracketed by HIP events recorded on its
 * stream.  dg_timing_read synchronises on the last event, returns the summed
 * device milliseconds and launch counts per kernel kind since the last read
 * (host pointers, any may be NULL) and resets them.  At most 16384 launches
 * are recorded between reads; later ones are counted in *dropped. */
dg_status dg_timing_enable(dg_ctx *ctx, int on);
dg_status dg_timing_read(dg_ctx *ctx, double *face_ms, long long *face_n, double *vol_ms, long long *vol_n,
                         double *cfl_ms, long long *cfl_n, long long *dropped);

/* ---------------------------------------------------------------------------
 * Batched ensembles: many independent boxes (own mesh size and order, same
 * dimension and physics) advanced together.  Boxes under 65536 cells are
 * grouped by order; each group runs one grouped launch per kernel kind and RK
 * stage over all of its boxes (a device table maps flat blocks to (box,
 * tile)); larger boxes run their own kernels (they fill the device alone).
 * The whole step of every box is captured once into a hipGraph and replayed.
 * Every box gives the same bits as stepping it alone with dg_step_cfl.
 * ------------------------------------------------------------------------- */
typedef struct dg_batch dg_batch;

/* nbox boxes, meshes[i] / orders[i] per box (same dim for all; each box
 * validated as by dg_init).  gamma, nu, kappa as dg_init; av must be NULL or
 * disabled (DG_EUNSUPPORTED otherwise).  Allocates every box's registers. */
dg_status dg_batch_init(int nbox, const dg_mesh *meshes, const int *orders, double gamma, double nu, double kappa,
                        const dg_av_params *av, const dg_options *opt, dg_batch **out);
void dg_batch_free(dg_batch *b);

/* One SSP-RK step of every box i (its own scheme by order), in place on the
 * device arrays w[i] (host array of nbox device pointers), each with its own
 * CFL time step computed on the device (eq. timestep).  The first call (and
 * any call with different pointers) captures the step into a hipGraph on
 * `stream`; later calls replay it.  use_graph = 0 launches the same grouped
 * kernels without a graph. */
dg_status dg_batch_step(dg_batch *b, double *const *w, int use_graph, void *stream);

/* The same step with caller-given step sizes: box i advances by dt_dev[i]
 * (device array of nbox doubles, 8-byte aligned, read on the device when the
 * step runs, so a captured graph replays with whatever values the array
 * holds then) instead of its CFL step.  A different dt_dev pointer, or
 * alternating with dg_batch_step, captures the graph again.  dg_batch_dt
 * then reports these values. */
dg_status dg_batch_step_dt(dg_batch *b, double *const *w, const double *dt_dev, int use_graph, void *stream);

/* Per-box step sizes of the last batched step (host array of nbox doubles).
 * Synchronises `stream`. */
dg_status dg_batch_dt(dg_batch *b, double *dt_out, void *stream);

/* Number of boxes of the batch (0 for NULL). */
int dg_batch_size(const dg_batch *b);

/* The context of box i (e.g. for per-box dg_step_cfl launches on the same
 * buffers, dg_rhs, totals).  Owned by the batch. */
dg_status dg_batch_box(dg_batch *b, int i, dg_ctx **ctx);

const char *dg_status_str(dg_status s);

#ifdef __cplusplus
}
#endif

#endif /* DG_H */
