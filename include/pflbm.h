/*
 * pflbm.h -- C ABI of the MI355X (gfx950) coupled phase-field lattice Boltzmann step.
 *
 * The method is the conservative Allen-Cahn phase-field LBM compared in
 * Schwarzmeier et al., "Comparison of free-surface and conservative
 * Allen-Cahn phase-field lattice Boltzmann method" (arXiv:2206.11637),
 * sec. "Conservative Allen-Cahn model":
 *   - phase-field PDFs h_i on D3Q15 (eq. lb_interface), phi = sum_i h_i
 *     (eq. zeroth_moment_phase), relaxation time tau_phi = M / c_s^2
 *     (eq. pflbm-tau), counter-term F^phi = 4 phi (1 - phi)/xi n applied with
 *     Guo forcing;
 *   - hydrodynamic PDFs g_i on D3Q27 (velocity-based, incompressible
 *     equilibrium eq. feq with rho_0 = 1), p* = sum_i g_i
 *     (eq. zeroth_moment_hydro), total force F = F_s + F_b + F_p + F_mu with
 *     F_s = mu_phi grad phi, F_b = rho g, F_p = -p* c_s^2 (rho_H - rho_L) grad phi,
 *     F_mu = nu (rho_H - rho_L) [grad u + grad u^T] grad phi taken from
 *     non-equilibrium moments; rho(phi) and tau(phi) linear in phi;
 *   - weighted-orthogonal MRT (eq. mrt) or BGK (eq. BGK) collisions,
 *     streaming (eq. streaming) with halfway bounce-back walls.
 *
 * Conventions for every entry point:
 *   - Lattice units: dx = dt = 1, c_s^2 = 1/3.
 *   - Grid: nx * ny * nz cells, cell index idx = x + nx * (y + ny * z).
 *     Scalar fields are N = nx*ny*nz values in that order; vector fields are
 *     three such planes (x, y, z components).  Populations are
 *     structure-of-arrays: population i of cell idx at [i * N + idx].
 *   - Non-periodic axes carry halfway bounce-back walls on the box faces; a
 *     solid mask (1 = solid) adds interior solids.  A solid or out-of-box
 *     neighbour contributes the cell's own phi to the grad/lap stencils.
 *   - Memory: the caller owns every device buffer, including the workspace
 *     the context lives in.  The library never allocates device memory and
 *     never frees caller memory.  Pointers passed in must stay valid while
 *     the context uses them.  "d_" marks device pointers, "host" host ones.
 *   - Streams: all work is enqueued on the stream given at creation, in
 *     order.  Only pflbm_reduce, pflbm_adjoint_grads and pflbm_sync wait
 *     for the stream.
 *   - Errors: every call returns a pflbm_status; nothing aborts.  Invalid
 *     arguments return PFLBM_ERR_ARG with no work enqueued.  HIP launch or
 *     runtime errors return PFLBM_ERR_HIP.  pflbm_last_error() holds a message.
 *   - Threads: one context must not be used from two threads at once.
 */
#ifndef PFLBM_H
#define PFLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pflbm_ctx pflbm_ctx;

typedef enum {
  PFLBM_OK = 0,
  PFLBM_ERR_ARG = 1,         /* invalid argument; nothing was enqueued            */
  PFLBM_ERR_STATE = 2,       /* call not valid in the context's current state     */
  PFLBM_ERR_HIP = 3,         /* HIP runtime or launch error                       */
  PFLBM_ERR_UNSTABLE = 4,    /* a reduction returned NaN/Inf                      */
  PFLBM_ERR_UNSUPPORTED = 5  /* combination of options not built                  */
} pflbm_status;

typedef enum {
  PFLBM_FP64 = 0,        /* FP64 populations, FP64 arithmetic                     */
  PFLBM_FP32 = 1,        /* FP32 populations, FP32 arithmetic                     */
  PFLBM_FP32_FP16S = 2   /* FP32 arithmetic, populations stored as FP16 of
                            value * 2^k, k per lattice from fp16_scale_log2      */
  /* Both FP32-arithmetic forms store h shifted: a slot holds h_i - w_i phi^n(r)
     with r the cell that reads it in the next step, and the collision works on
     deviations from w_i phi^{n-1} of the cell (rounding then acts on the
     per-step change, not on h ~ w_i); g is stored unshifted.  FP64 stores plain
     values. */
} pflbm_precision;

typedef enum { PFLBM_BGK = 0, PFLBM_MRT = 1 } pflbm_collision;

/* Streaming scheme (paper: streaming eq.; both give the same results):
 *   PFLBM_STREAM_AB: two population buffers read in pull form; one fused
 *     kernel per step also forms phi (fastest; twice the population memory);
 *   PFLBM_STREAM_AA: the in-place AA pattern, one population buffer; each
 *     step is a collide-and-stream kernel plus a light phi pass. */
typedef enum { PFLBM_STREAM_AB = 0, PFLBM_STREAM_AA = 1 } pflbm_streaming;

/* Source term of the hydrodynamic collision (the paper applies the forces
 * with Guo's scheme in collision space, sec. "Lattice Boltzmann equations"):
 *   PFLBM_FORCING_FIRST: 3 w_i c_i.F / rho, the first-order part (default);
 *   PFLBM_FORCING_GUO:   Guo's full term w_i [3 (c_i - u) + 9 (c_i.u) c_i].F / rho,
 *                        whose second moment (u F^T + F u^T)/rho removes the
 *                        force's error term from the stress.
 * Both are applied with the (I - S/2) factor of the collision's rates. */
typedef enum { PFLBM_FORCING_FIRST = 0, PFLBM_FORCING_GUO = 1 } pflbm_forcing;

typedef struct {
  int32_t nx, ny, nz;     /* cells per axis, each >= 1                            */
  uint32_t periodic;      /* bit0 x, bit1 y, bit2 z; clear bit = walls on that axis */
  int32_t precision;      /* pflbm_precision                                      */
  int32_t collision;      /* pflbm_collision                                      */
  int32_t has_mask;       /* 1: pflbm_set_mask must be called before init          */
  int32_t streaming;      /* pflbm_streaming                                      */
  int32_t forcing;        /* pflbm_forcing                                        */
} pflbm_desc;

typedef struct {
  double tau_H, tau_L;    /* hydrodynamic relaxation times (> 1/2); nu = (tau - 1/2)/3,
                             tau(phi) = tau_L + phi (tau_H - tau_L)                */
  double mobility;        /* M > 0; phase-field rate omega_phi = 1 / (3 M + 1/2)   */
  double xi;              /* interface width > 0; +inf switches the counter-term
                             and the chemical potential off                        */
  double sigma;           /* surface tension >= 0; mu_phi = 4 beta phi (phi-1)(phi-1/2)
                             - kappa lap phi, beta = 12 sigma/xi, kappa = 3 sigma xi/2 */
  double rho_H, rho_L;    /* heavy / light densities (> 0); rho(phi) linear        */
  double g[3];            /* body acceleration                                     */
  double s_high;          /* MRT rate of moments of degree >= 3 (0 < s < 2)        */
  double fp16_scale_log2[2]; /* FP16S storage exponents k for h and g (integers,
                             |k| <= 24); ignored by the other precisions          */
  double normal_eps;      /* > 0: n = grad phi / sqrt(|grad phi|^2 + eps^2).  The
                             paper leaves n undefined where grad phi = 0; 1e-4
                             only touches cells many widths from an interface and
                             keeps the reverse mode well conditioned              */
  double s_bulk;          /* MRT rate of the bulk mode of g (the trace of its
                             second-order moments, polynomial |c|^2 - 1): 0 = the
                             second-order rate omega(phi) (default), else in (0, 2).
                             The viscous force F_mu then recovers the trace part of
                             the strain rate with this rate.  Ignored by BGK      */
  double rho_g_ref;       /* body force F_b = (rho(phi) - rho_g_ref) g.  0 (default):
                             gravity on the whole density, as written in the paper;
                             rho_H: its buoyant part only, the heavy phase's
                             hydrostatic pressure taken into p (the same flow in
                             the incompressible limit, with p* of a rising light
                             phase no longer drifting with its height); finite  */
} pflbm_params;

/* Bytes of device workspace for a context with this description (256-aligned
 * regions: one (AA) or two (AB) population buffers, two phi buffers, the mask
 * and its neighbour bits, reduction partials).  Returns 0 if the description
 * is invalid: an enum out of range, an axis < 1, N = nx ny nz >= 2^29 (FP32
 * and FP16 storage) or >= 2^28 (FP64) -- the population offsets within one
 * opposite pair are 32-bit byte offsets -- or a shape so thin that its tiles
 * (16-64 cells wide, 256 cells each) times nz reach 2^24 blocks. */
size_t pflbm_workspace_bytes(const pflbm_desc* desc);

/* Creates a host-side context that uses d_workspace (>= pflbm_workspace_bytes,
 * 256-byte aligned) and enqueues everything on hip_stream (a hipStream_t, NULL =
 * the null stream).  Parameters default to those of a capillary-wave case
 * until pflbm_set_params is called.  *out receives the context. */
pflbm_status pflbm_create(const pflbm_desc* desc, void* d_workspace, size_t bytes,
                          void* hip_stream, pflbm_ctx** out);

/* Frees the host-side context only (the workspace stays the caller's). */
pflbm_status pflbm_destroy(pflbm_ctx* ctx);

/* Validates and sets the physical parameters (tau > 1/2, M > 0, xi > 0,
 * sigma >= 0, rho > 0, 0 < s_high < 2, normal_eps > 0, s_bulk = 0 or in
 * (0, 2), rho_g_ref finite).  Takes effect for the next step.  With FP16
 * storage, fp16_scale_log2 is part of the stored state's encoding: once the
 * state is initialised (or loaded) a different value returns PFLBM_ERR_STATE
 * and changes nothing; saved states must be loaded into contexts with the
 * scale they were written with. */
pflbm_status pflbm_set_params(pflbm_ctx* ctx, const pflbm_params* params);

/* Copies an N-byte solid mask (1 = solid, 0 = fluid) into the workspace
 * (device-to-device, asynchronous) and derives each cell's solid-neighbour
 * bits from it.  Only for contexts created with has_mask. */
pflbm_status pflbm_set_mask(pflbm_ctx* ctx, const uint8_t* d_solid);

/* Equilibrium initialisation (sec. "Lattice Boltzmann equations", eq. feq with
 * rho_0 = 1 for g, and the phase field's equilibrium phi Gamma_i(u) for h; the
 * initial phase field is the caller's, e.g. the tanh profile of sec.
 * "Numerical experiments"): h_i = phi0 w_i [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u],
 * g_i = w_i [p*0 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u], zero in solids, then
 * phi = sum_i h_i (eq. zeroth_moment_phase).  d_phi0 [N], d_u0 [3][N],
 * d_pstar0 [N] (FP64; d_u0 or d_pstar0 may be NULL for zero).  Resets the
 * step counter to 0. */
pflbm_status pflbm_init_equilibrium(pflbm_ctx* ctx, const double* d_phi0,
                                    const double* d_u0, const double* d_pstar0);

/* Advances nsteps >= 0 time steps, asynchronously.  One step is the coupled
 * update of sec. "Lattice Boltzmann equations": the phase-field LBE with the
 * counter-term source (eq. lb_interface, relaxation eq. pflbm-tau), the
 * hydrodynamic LBE with F = F_s + F_b + F_p + F_mu, both collided with
 * eq. mrt (or eq. BGK) and streamed (eq. streaming) with halfway bounce-back,
 * then phi = sum_i h_i (eq. zeroth_moment_phase).  With a check interval
 * K > 0 (pflbm_set_check_interval) it also reduces sum(phi) and sum(p*) in
 * FP64 every K steps, waits for that result, and stops with
 * PFLBM_ERR_UNSTABLE at the first non-finite one; the step count then names
 * the step after which it was detected. */
pflbm_status pflbm_step(pflbm_ctx* ctx, int64_t nsteps);

/* Sets the stability check interval K of pflbm_step (0 = never, the
 * default; each check costs one reduction and one host round trip). */
pflbm_status pflbm_set_check_interval(pflbm_ctx* ctx, int64_t every);

/* Cell moments of the current state as FP64 (sec. "Lattice Boltzmann
 * equations": phi = sum_i h_i, eq. zeroth_moment_phase; p* = sum_i g_i,
 * eq. zeroth_moment_hydro, the pressure being p = p* rho c_s^2; u from the
 * first moment of g with half the force): phi [N], u [3][N] (the
 * force-corrected velocity u = j + F/(2 rho)), p* [N]; zero in solids.  Any
 * output may be NULL. */
pflbm_status pflbm_read_moments(pflbm_ctx* ctx, double* d_phi, double* d_u, double* d_pstar);

/* The current phase field phi^n = sum_i h_i^n as FP64 [N] (cheap; no forces). */
pflbm_status pflbm_read_phi(pflbm_ctx* ctx, double* d_phi);

/* Post-streaming populations in natural order, decoded to FP64:
 * d_h [15][N], d_g [27][N] in the library's velocity order (pflbm_lattice). */
pflbm_status pflbm_read_populations(pflbm_ctx* ctx, double* d_h, double* d_g);

/* FP64 sums over fluid cells of the moments of sec. "Lattice Boltzmann
 * equations" (the phase mass the conservative Allen-Cahn model conserves, the
 * sum of p* and the momentum): out_host = {sum phi, sum p*, sum j_x, sum j_y,
 * sum j_z} with j = sum_i c_i g_i.  Deterministic (fixed reduction order).
 * Waits for the stream.  Returns PFLBM_ERR_UNSTABLE if any is NaN/Inf. */
pflbm_status pflbm_reduce(pflbm_ctx* ctx, double out_host[5]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sums of
 * pflbm_reduce with its per-block partial sums kept in a static device array
 * of the library (16 MiB per GPU, held until the process ends) instead of the
 * context's workspace; same results, bitwise.  Returns PFLBM_ERR_ARG when the
 * lattice needs more than that: 40 bytes per tile and z plane (tiles of 256
 * cells, 64 x 4 where nx > 32), rounded up to 256, plus 256, i.e. about
 * 1.3 MB for 128x512x128 and 8.8 MB for 384^3.  Allocates nothing.  Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU (two host
 * threads, or contexts on different streams of the same GPU) race.  Waits for
 * the stream. */
pflbm_status pflbm_reduce_static(pflbm_ctx* ctx, double out_host[5]);

/* Bytes of one saved state: h [15][N] and g [27][N] in storage precision
 * (layout of the streaming scheme), phi^n [N] and, for the FP32 and FP16S
 * forms, phi^{n-1} [N] (the shift reference; defined on fluid cells). */
size_t pflbm_state_bytes(const pflbm_ctx* ctx);

/* Copies the state to / from d_buf (device-to-device, asynchronous).  The
 * step count is not part of the buffer: load takes it explicitly (with
 * PFLBM_STREAM_AA its parity selects the layout). */
pflbm_status pflbm_save_state(pflbm_ctx* ctx, void* d_dst);
pflbm_status pflbm_load_state(pflbm_ctx* ctx, const void* d_src, int64_t step_count);

/* One time step from a saved state of level n (d_src, as written by
 * pflbm_save_state) into another, non-overlapping buffer of the same size
 * (d_dst, level n + 1), without touching the context's own state; used to
 * recompute checkpoint segments without copies.  Asynchronous.
 * flags (PFLBM_STREAM_AB contexts only; PFLBM_ERR_ARG otherwise), for a chain
 * of such steps:
 *   PFLBM_STATES_WRITE_SRC_PHI  the step also writes the phi^n it forms into
 *                               d_src's phi^n slot (d_src is then written);
 *   PFLBM_STATES_SKIP_DST_PHI   d_dst's phi^{n+1} slot is left unformed (a
 *                               following step from d_dst with
 *                               PFLBM_STATES_WRITE_SRC_PHI fills it); saves one
 *                               pass over h per step.
 * Without flags d_src is only read and d_dst is complete. */
#define PFLBM_STATES_WRITE_SRC_PHI 1
#define PFLBM_STATES_SKIP_DST_PHI 2
pflbm_status pflbm_step_states(pflbm_ctx* ctx, void* d_src, void* d_dst, int64_t n, int32_t flags);

/* Steps taken since the last init or load. */
int64_t pflbm_step_count(const pflbm_ctx* ctx);

/* Advances nsteps like pflbm_step while timing every kernel with HIP events
 * recorded on the context's stream between consecutive launches (no host
 * synchronisation inside the loop); out_ms_host receives {summed durations of
 * the collide-and-stream kernel, summed durations of the phi-update kernel
 * (0 with PFLBM_STREAM_AB, whose step kernel forms phi itself), total elapsed
 * time} in milliseconds.  Waits for the stream at the end. */
pflbm_status pflbm_profile_step(pflbm_ctx* ctx, int64_t nsteps, double out_ms_host[3]);

/* Waits for all work on the context's stream. */
pflbm_status pflbm_sync(pflbm_ctx* ctx);

/* Host copy of the library's velocity set for q = pflbm_phase_q() (the phase
 * field's) or 27 (the hydrodynamics'): c_out [q][3] integers, w_out [q]
 * weights.  Either may be NULL. */
pflbm_status pflbm_lattice(int32_t q, int32_t* c_out, double* w_out);

/* Velocity count of this library's phase lattice: 15 (D3Q15, libpflbm.so) or
 * 27 (D3Q27, the velocity set the paper uses for both lattices in 3D:
 * libpflbm_d3q27.so, the same interface built with PFLBM_PHASE_D3Q27).  Every
 * "[15][N]" phase-field array of this interface has pflbm_phase_q() rows. */
int32_t pflbm_phase_q(void);

/* ---------------------------------------------------------------------------
 * Reverse mode (adjoint) of the step, for gradients of a loss of the phase
 * field with respect to the mobility M, the surface tension sigma, the
 * interface width xi and the initial phase field phi0.  The adjoint state
 * lambda holds dL/dh and dL/dg of one time level.  Arithmetic is FP64 for
 * PFLBM_FP64 contexts and FP32 otherwise; the parameter gradients are
 * accumulated in FP64.  With FP16S storage the quantisation is treated as the
 * identity.
 * ------------------------------------------------------------------------- */

/* Bytes of the adjoint workspace for this description (0 if invalid). */
size_t pflbm_adjoint_workspace_bytes(const pflbm_desc* desc);

/* Attaches an adjoint workspace and clears lambda and the gradient sums. */
pflbm_status pflbm_adjoint_attach(pflbm_ctx* ctx, void* d_adj_workspace, size_t bytes);

/* Clears lambda and the gradient sums (start of a new backward pass). */
pflbm_status pflbm_adjoint_reset(pflbm_ctx* ctx);

/* Adds dL/dphi^n (FP64 [N], the loss's direct sensitivity to the phase field
 * of the current adjoint time level n) into lambda. */
pflbm_status pflbm_adjoint_inject_phi(pflbm_ctx* ctx, const double* d_dl_dphi);

/* One reverse step: lambda^{n+1} -> lambda^n through the step n -> n+1,
 * using the primal state of level n (a buffer written by pflbm_save_state
 * when the step count was n, or by pflbm_step_states with its phi^n formed),
 * and adds this step's contributions to dL/dM and dL/dsigma. */
pflbm_status pflbm_adjoint_step(pflbm_ctx* ctx, const void* d_state_n, int64_t n);

/* Reverse of pflbm_init_equilibrium for phi0: d_dphi0 [N] (FP64) receives
 * dL/dphi0 = sum_i lambda_h,i Gamma_i(u0), with u0 (FP64 [3][N], NULL = 0)
 * the velocity the state was initialised with; zero in solids. */
pflbm_status pflbm_adjoint_init(pflbm_ctx* ctx, const double* d_u0, double* d_dphi0);

/* out_host = {dL/dM, dL/dsigma, dL/dxi} accumulated since attach/reset (the
 * mobility, surface tension and interface width of sec. "Conservative
 * Allen-Cahn model": M sets the phase-field relaxation, eq. pflbm-tau; sigma
 * and xi set the chemical potential's beta = 12 sigma/xi and kappa =
 * 3 sigma xi/2, and xi the counter-term 4 phi (1 - phi)/xi).  dL/dxi holds phi0
 * fixed: a phi0 built from xi adds dL/dphi0 . dphi0/dxi.  Waits for the
 * stream. */
pflbm_status pflbm_adjoint_grads(pflbm_ctx* ctx, double out_host[3]);

/* ---------------------------------------------------------------------------
 * Halo pack of a z-slab decomposition (the part of the multi-GPU step that one
 * GPU can run).  With the lattice split into slabs along z, each step pulls
 * across a slab face exactly the populations that the streaming step (paper
 * sec. "Lattice Boltzmann equations", eq. streaming) moves from one plane to
 * the next along z: those with c_z = -1 stored at plane 0 (bound for the slab
 * below) and those with c_z = +1 stored at plane nz - 1 (bound for the slab
 * above).  Copies them from the current state into d_dst on the context's
 * stream, asynchronously.  Layout of d_dst: face 0 (plane 0, c_z = -1) then
 * face 1 (plane nz - 1, c_z = +1); within a face first the h rows, then the g
 * rows, each in the direction order of pflbm_lattice / pflbm_phase_q; a row is
 * the nx * ny values of one population on that plane, x fastest, in the
 * storage type exactly as the state holds them (FP64, FP32, or FP16 with its
 * scale and shift, as in a saved state).  Rows per face: 5 + 9 (D3Q15 phase
 * lattice) or 9 + 9 (D3Q27).  *bytes_needed (required) receives the size
 * 2 x rows x nx x ny x storage size; with d_dst NULL nothing else happens.
 * d_dst is device memory owned by the caller, aligned to the storage size.
 * Returns PFLBM_ERR_ARG for a NULL bytes_needed, a misaligned d_dst or
 * dst_bytes below the size, PFLBM_ERR_STATE without an initialised state or
 * with PFLBM_STREAM_AA (whose slots depend on the step parity; only the
 * two-buffer scheme is packed).
 * ------------------------------------------------------------------------- */
pflbm_status pflbm_pack_faces(pflbm_ctx* ctx, void* d_dst, size_t dst_bytes, size_t* bytes_needed);

/* ---------------------------------------------------------------------------
 * Measurement helper (not part of the method): the HBM ceiling of a kernel
 * that only streams data.  Copies `bytes` from d_src to d_dst (device memory,
 * both 16-byte aligned, not overlapping, bytes a multiple of 16) on
 * hip_stream, asynchronously, with one of these kernels:
 *   PFLBM_COPY_W4          4-byte accesses, 8 per thread, non-temporal
 *   PFLBM_COPY_W16         16-byte accesses, 4 per thread, non-temporal
 *   PFLBM_COPY_W16_CACHED  16-byte accesses, 4 per thread, cached
 *   PFLBM_COPY_SOA43       the step kernel's access pattern without its
 *                          arithmetic: bytes = 43 rows of N floats (42
 *                          populations + the phase field); one thread per cell
 *                          loads its 43 values (cached, all in flight) and
 *                          stores them to the same rows of d_dst (non-temporal)
 *   PFLBM_COPY_SOA43_NT    the same with non-temporal loads
 *   PFLBM_COPY_SOA43_F64, PFLBM_COPY_SOA43_F64_NT
 *                          the same two with 43 rows of N doubles (the FP64
 *                          step's pattern)
 * Returns PFLBM_ERR_ARG for a bad pointer, size or form (nothing enqueued).
 * ------------------------------------------------------------------------- */
enum {
  PFLBM_COPY_W4 = 0,
  PFLBM_COPY_W16 = 1,
  PFLBM_COPY_W16_CACHED = 2,
  PFLBM_COPY_SOA43 = 3,
  PFLBM_COPY_SOA43_NT = 4,
  PFLBM_COPY_SOA43_F64 = 5,
  PFLBM_COPY_SOA43_F64_NT = 6
};
pflbm_status pflbm_hbm_copy(const void* d_src, void* d_dst, size_t bytes, int32_t form, void* hip_stream);

const char* pflbm_status_string(pflbm_status s);
const char* pflbm_last_error(const pflbm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* PFLBM_H */
