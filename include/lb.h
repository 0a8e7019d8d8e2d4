/*
 * lb.h -- C ABI of the MI355X D3Q19 lattice-Boltzmann library (liblb.so).
 *
 * The operation is the per-site lattice-Boltzmann update the paper
 * benchmarks (Section IV: an LB collision for a mixture of two fluids,
 * inner loops over the 19 lattice momenta and the 3 dimensions, double
 * precision lattice fields), followed by periodic propagation.  The paper
 * gives no formula; the library implements the standard readings:
 *
 *   single fluid  f*_i = f_i - (f_i - f^eq_i(rho, u)) / tau_f
 *   binary fluid  f*_i = f_i - (f_i - f^eq_i(rho, u, P)) / tau_f
 *                 g*_i = g_i - (g_i - g^eq_i(phi, u, mu)) / tau_g
 *   propagation   f_i(s + c_i) <- f*_i(s)   (periodic in x, y, z)
 *
 * with rho = sum f_i, u = sum f_i c_i / rho, phi = sum g_i,
 *   mu   = A phi + B phi^3 - kappa lap(phi),
 *   P_ab = [A/2 phi^2 + 3B/4 phi^4 - kappa phi lap(phi) - kappa/2 |grad phi|^2] d_ab
 *          + kappa d_a phi d_b phi,
 *   f^eq_i = w_i {rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u] + 9/2 [c_i.P.c_i - tr P / 3]},
 *   g^eq_i = w_i {phi [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u] + 9/2 (gamma mu - phi/3)(|c_i|^2 - 1)},
 *   tau_g  = mobility / gamma + 1/2,
 * grad and lap by second-order 7-point central differences (the paper's
 * application solves its order parameter by finite differences, Section
 * II-A).
 *
 * Velocity ordering (i = 0..18): rest first, then the 18 velocities with
 * |c|^2 in {1,2} in lexicographic order of (c_x, c_y, c_z):
 *   1 (-1,-1,0)  2 (-1,0,-1)  3 (-1,0,0)  4 (-1,0,1)  5 (-1,1,0)  6 (0,-1,-1)
 *   7 (0,-1,0)   8 (0,-1,1)   9 (0,0,-1) 10 (0,0,1)  11 (0,1,-1) 12 (0,1,0)
 *  13 (0,1,1)   14 (1,-1,0)  15 (1,0,-1) 16 (1,0,0)  17 (1,0,1)  18 (1,1,0)
 * weights 1/3 (rest), 1/18 (|c|^2 = 1), 1/36 (|c|^2 = 2).
 *
 * Layout (Section III-B, structure of arrays): site s = x + nx*(y + ny*z);
 * a distribution in "canonical" layout is 19 arrays of N = nx*ny*nz values,
 * direction-major, i.e. element (i, s) at offset i*N + s.  Vector moments
 * are component-major: u[a*N + s], a = x, y, z.
 *
 * Memory and streams.  Every pointer passed to a liblb.so function is a
 * DEVICE pointer unless stated otherwise.  The caller owns all memory: the
 * workspace given to lb_create and every input/output array (the one
 * exception is the library's fixed device array behind the allocation-free
 * lb_conserved_sums_noalloc).  All calls
 * that touch device memory are asynchronous on the context's stream and
 * never synchronise the device (the exceptions are lb_kernel_times, which
 * waits for the events it reads, and lb_destroy, which waits for the
 * stream).  Kernel launch failures return LB_EDEVICE; faults inside a
 * kernel surface at the caller's next synchronisation.  A context is not
 * thread-safe.  Invalid arguments are detected before any work is queued
 * and leave the context unchanged.
 *
 * The target copy of the lattice is the master copy (Section III-A): the
 * host sees the state only through lb_moments, lb_get_state and
 * lb_conserved_sums.
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes.  Every function returns one of these (lb_strerror aside). */
#define LB_OK        0
#define LB_EINVAL   (-1)   /* bad argument: NULL pointer, size, parameter range, wrong model */
#define LB_ENOMEM   (-2)   /* workspace smaller than lb_workspace_bytes() */
#define LB_EDEVICE  (-3)   /* a HIP runtime call or kernel launch failed */
#define LB_ENOTSUP  (-4)   /* valid request this build does not implement */
#define LB_ERANGE   (-5)   /* lattice too large for the fixed scratch of an allocation-free call */

/* Models. */
#define LB_SINGLE   0      /* one fluid, distribution f */
#define LB_BINARY   1      /* binary mixture, distributions f and g (g carries phi) */

/* Collision of f (either model; g always relaxes with 1/tau_g).  LB_TRT:
 * two-relaxation-time collision (the
 * parts of f - f^eq even and odd under c -> -c relax with 1/tau_f and
 * 1/tau_minus; tau_minus = tau_f is BGK).  LB_MRT: multiple-relaxation-time
 * collision in the orthogonal moment basis of d'Humieres et al. (2002): the
 * shear stresses relax with 1/tau_f, the energy fluxes with 1/tau_minus, the
 * energy moment with 1/tau_bulk (bulk viscosity (2/9)(tau_bulk - 1/2)), the
 * even ghosts (eps, pi_xx, pi_ww) with 1/tau_ghost_even and the odd ghosts
 * (m_x, m_y, m_z) with 1/tau_ghost_odd; tau_bulk = tau_ghost_even = tau_f and
 * tau_ghost_odd = tau_minus is LB_TRT.  Neither is part of the paper's
 * benchmark, which does not say which collision it uses (Section IV). */
#define LB_BGK      0
#define LB_TRT      1
#define LB_MRT      2

/* The binary step's kernel.  LB_STEP_MARCH: one single-pass kernel that
 * marches each tile column through a chunk of z planes, computing phi and its
 * stencils on chip (608 B/site in FP64): fastest on large lattices.
 * LB_STEP_TWO_PASS: a phi pass, then the fused collide (776 B/site), every
 * site in parallel: fastest on small lattices, where the march has too few
 * blocks to hide its per-plane latency.  LB_STEP_AUTO (0, the default): the
 * march when its grid has at least 256 blocks (64 x 8 tiles; chunks of 64
 * planes where that gives more than 512 blocks, else as many chunks as fill 512
 * blocks, at most nz/16 of them; 128^3 has 256), else the
 * two-pass step.  (FP32 and FP16 march on 128 x 4 tiles where nx mod 128 is
 * 0 or above 64.) */
#define LB_STEP_AUTO     0
#define LB_STEP_MARCH    1
#define LB_STEP_TWO_PASS 2

/* Storage precision of the distributions.
 * LB_F64: f and g stored as IEEE double, FP64 arithmetic, stored directly.
 * LB_F32: stored as float deviations d_i = f_i - w_i*rho0 (g: g_i - w_i*phi0),
 *         FP32 arithmetic written in deviation form.
 * LB_F16: as LB_F32 but stored as IEEE binary16 (round to nearest even). */
#define LB_F64      0
#define LB_F32      1
#define LB_F16      2

typedef struct lb_params {
    int32_t nx, ny, nz;   /* periodic extents, each >= 1, nx*ny*nz < 2^29     */
    int32_t model;        /* LB_SINGLE or LB_BINARY                           */
    int32_t storage;      /* LB_F64, LB_F32 or LB_F16                          */
    int32_t vvl;          /* sites per lane along z of the fused collide and phi
                             kernels (the virtual vector length of the targetDP
                             execution model, Section III-C): 0 or 1 (default), 2, 4 */
    int32_t collision;    /* LB_BGK (default), LB_TRT or LB_MRT               */
    int32_t binary_step;  /* LB_BINARY: which step kernel runs (LB_STEP_*); the
                             two give the same bits; ignored for LB_SINGLE     */
    double  tau_f;        /* BGK relaxation time of f, > 0.5                  */
    double  A, B, kappa;  /* free energy (binary only); kappa >= 0            */
    double  mobility;     /* Cahn-Hilliard mobility M > 0 (binary only)       */
    double  gamma;        /* mobility parameter Gamma > 0 (binary only)       */
    double  rho0, phi0;   /* deviation references for LB_F32/LB_F16; ignored for LB_F64 */
    double  tau_minus;    /* LB_TRT: relaxation time of the odd part; LB_MRT: of the
                             energy fluxes; > 0.5                              */
    double  tau_bulk;     /* LB_MRT: energy moment (bulk viscosity), > 0.5     */
    double  tau_ghost_even; /* LB_MRT: eps, pi_xx, pi_ww, > 0.5                */
    double  tau_ghost_odd;  /* LB_MRT: m_x, m_y, m_z, > 0.5                    */
} lb_params;

typedef struct lb_ctx lb_ctx;   /* opaque; created by lb_create */

/* Bytes of device workspace a context with these parameters needs.
 * Host-only (touches no device).  LB_EINVAL on bad parameters.
 * Paper: Section III-B (targetMalloc: target lattice data is allocated with
 * error checking); here the caller allocates and the library only sizes. */
int lb_workspace_bytes(const lb_params* p, size_t* bytes);

/* Create a context.  `workspace` is a device allocation of at least
 * lb_workspace_bytes() bytes, 256-byte aligned, owned by the caller and
 * borrowed until lb_destroy; `stream` is a hipStream_t (NULL = the null
 * stream).  Queues no device work.  *out receives the context.
 * Paper: Section III-A (the target holds the master copy of the lattice
 * data) and Section III-B (lattice fields on the target, structure of
 * arrays).  LB_EINVAL on bad parameters or a NULL workspace, LB_ENOMEM if
 * workspace_bytes is too small; nothing is created then. */
int lb_create(const lb_params* p, void* workspace, size_t workspace_bytes,
              void* stream, lb_ctx** out);

/* Change the stream subsequent calls are queued on.  Not in the paper
 * (its CUDA layer synchronises after every launch, Section III-C's
 * syncTarget; here ordering is the caller's stream). */
int lb_set_stream(lb_ctx* ctx, void* stream);

/* Set the state to equilibrium: f = f^eq(rho, u[, P(phi)]) and, for the
 * binary model, g = g^eq(phi, u, mu(phi)), the stencils applied to the given
 * phi.  rho[N], u[3*N] component-major, phi[N] (NULL for LB_SINGLE), all
 * FP64 device arrays in site order.  The state becomes the pre-collision
 * state at t = 0.  Paper: Section III-B (copyToTarget: lattice data enters
 * the target once, as whole-lattice fields) and Section IV (the benchmark's
 * two-fluid lattice-Boltzmann model; the equilibria are the readings in the
 * file header).  LB_EINVAL if rho or u is NULL, or phi is NULL for
 * LB_BINARY / not NULL for LB_SINGLE. */
int lb_init_equilibrium(lb_ctx* ctx, const double* rho, const double* u, const double* phi);

/* One collision of every site of the current state (binary: computes phi,
 * its stencils, mu and P from the current g first).  Paper: Section IV (the
 * benchmarked operation: a lattice-Boltzmann collision of a two-fluid
 * mixture, loops over 19 momenta and 3 dimensions) and Section II-A (the
 * order parameter's gradients by finite differences).  LB_EINVAL on NULL. */
int lb_collide(lb_ctx* ctx);

/* One periodic propagation f_i(s + c_i) <- f_i(s) of every population.
 * Paper: Section II-A (lattice-Boltzmann hydrodynamics on a regular
 * lattice); the paper benchmarks the collision alone, propagation is the
 * other half of the standard step.  On a state that is not pending this
 * only marks it pending (no kernel).  LB_EINVAL on NULL. */
int lb_propagate(lb_ctx* ctx);

/* nsteps x (collide; propagate).  nsteps == 0 is a no-op, < 0 is LB_EINVAL.
 * Each step is one launch of a fused pull-stream + collide kernel: for
 * LB_BINARY on large lattices the single-pass march, which sums phi from
 * the pulled g and takes its stencils on chip; on small lattices (or with
 * LB_STEP_TWO_PASS) a phi kernel, then the fused collide (see
 * binary_step).  Paper: Section IV (collision) and Section II-A
 * (propagation, finite-difference gradients of phi). */
int lb_step(lb_ctx* ctx, int32_t nsteps);

/* Moments of the current state, FP64: rho[N], u[3*N] component-major, and
 * phi[N] (binary only; NULL to skip).  rho or u may be NULL to skip them.
 * Paper: Section III-A (the host copy is refreshed from the target master
 * copy when needed) and Section III-B (copyFromTarget, structure-of-arrays
 * fields, a vector field as three components).  LB_EINVAL if phi is given
 * for LB_SINGLE. */
int lb_moments(lb_ctx* ctx, double* rho, double* u, double* phi);

/* out[5] (device, FP64) = (sum rho, sum j_x, sum j_y, sum j_z, sum phi) of
 * the current state, summed in a fixed order (bitwise reproducible for a
 * given lattice and state).  sum phi is 0 for LB_SINGLE.  Paper: Section V
 * (reductions over the lattice, which the paper leaves outside its layer);
 * uses the context's partial-sum area.  LB_EINVAL on NULL. */
int lb_conserved_sums(lb_ctx* ctx, double* out);

/* out[10] (device, FP64) = statistics of the current state, reduced in a
 * fixed order (device reductions; the paper lists reductions as future work
 * of its layer, Section V): 0 sum rho, 1-3 sum j, 4 sum phi, 5 sum rho u.u
 * (twice the kinetic energy), 6 min phi, 7 max phi, 8 sum phi^2, 9 max u.u.
 * Entries 4 and 6-8 are 0 for LB_SINGLE.  NaN anywhere in the state shows up
 * in the sums. */
int lb_field_stats(lb_ctx* ctx, double* out);

/* Copy the current state out / in, canonical layout, storage dtype (double,
 * float or binary16), deviations for LB_F32/LB_F16.  f has 19*N elements; g
 * likewise (binary only; NULL otherwise).  Paper: Section III-B
 * (copyFromTarget / copyToTarget of whole lattice fields; structure of
 * arrays, element (i, s) at i*N + s).  Device-to-device copies on the
 * stream.  LB_EINVAL if f is NULL or g does not match the model. */
int lb_get_state(lb_ctx* ctx, void* f, void* g);
int lb_set_state(lb_ctx* ctx, const void* f, const void* g);

/* Change tau_f (> 0.5) for subsequent collisions.  Not in the paper (a
 * kernel parameter, the role Section III-B gives to copyConstant...ToTarget).
 * LB_EINVAL if tau_f <= 0.5 or not finite. */
int lb_set_tau(lb_ctx* ctx, double tau_f);

/* nsteps x (collide; propagate) like lb_step (LB_SINGLE: any collision;
 * LB_BINARY: any collision), recording each step's
 * post-collision field (before its propagation) in caller memory, canonical
 * layout, storage dtype.  LB_SINGLE: step k (0-based) writes
 * post[k*19*N + i*N + s] (nsteps*19*N elements).  LB_BINARY: step k writes f*
 * at post[k*38*N + i*N + s] and g* at post[k*38*N + 19*N + i*N + s]
 * (nsteps*38*N elements); if phi is not NULL, phi[k*N + s] also receives the
 * order parameter of the state step k collides (compute dtype: double for
 * LB_F64, float otherwise).  phi must be NULL for LB_SINGLE.  The state
 * afterwards equals that after lb_step(nsteps).  Used by the adjoints'
 * segment recompute: post[k] holds the state of step k+1 in pending (pull)
 * form.  nsteps == 0 is a no-op.  Not in the paper (the forward half of the
 * checkpoint-and-recompute adjoint, which the paper does not have).
 * LB_EINVAL if post is NULL with nsteps > 0 or phi is given for LB_SINGLE. */
int lb_step_record(lb_ctx* ctx, int32_t nsteps, void* post, void* phi);

/* Adjoint (reverse) of one single-fluid step f^{n+1} = propagate(collide(f^n)),
 * LB_SINGLE + LB_F64 only, for the context's collision.  Every collision is
 * f* = f - Omega (f - f^eq(f)) with a constant symmetric Omega (BGK: I/tau_f;
 * TRT and MRT: the relaxation of lb_params' rate groups), so the adjoint is
 * lambda^n = lambda* - (I - J)^T Omega lambda*, J = d f^eq / d f.
 * f (19*N, canonical FP64) is f^n itself when
 * f_pending == 0, or the post-collision field of step n-1 (as written by
 * lb_step_record) when f_pending != 0, in which case f^n_i(s) = f_i(s - c_i).
 * lam_next[19*N] = dL/df^{n+1}, canonical FP64; lam_n[19*N] receives dL/df^n
 * (must not alias the inputs).  domega (device doubles) is INCREMENTED by
 * this step's dL/d(1/tau) for each relaxation time: 1 value for LB_BGK
 * (tau_f), 2 for LB_TRT (tau_f, tau_minus), 5 for LB_MRT (tau_f, tau_minus,
 * tau_bulk, tau_ghost_even, tau_ghost_odd); the caller zeroes them first and
 * converts with dL/dtau = -dL/domega / tau^2.  Uses the context's times.
 * Not in the paper (it has no adjoint); the transpose of the step of
 * lb_step.  LB_ENOTSUP for LB_BINARY or reduced storage; LB_EINVAL on NULL
 * or aliasing arrays. */
int lb_adjoint_step(lb_ctx* ctx, const double* f, int f_pending, const double* lam_next,
                    double* lam_n, double* domega);

/* Replace the physical parameters (tau_f, A, B, kappa, mobility, gamma,
 * tau_minus, tau_bulk, tau_ghost_even, tau_ghost_odd) for subsequent calls.
 * Every other field (sizes, model, storage, vvl, collision, binary_step,
 * rho0, phi0) must equal the context's, else LB_EINVAL; values are
 * validated as by lb_create.  The state is kept.  Not in the paper (the
 * operation's constant parameters, Section III-B's copyConstant family). */
int lb_set_params(lb_ctx* ctx, const lb_params* p);

/* Adjoint (reverse) of one binary-fluid step, LB_BINARY + LB_F64 only, for
 * f relaxing by any collision (g always relaxes by BGK).  The step is the one of lb_step: f and g relax to their equilibria, whose
 * pressure tensor and chemical potential read phi = sum g at the site and
 * its six neighbours (central-difference gradient and 7-point Laplacian,
 * Section II-A's finite-difference order-parameter model), then both
 * propagate.  f, g (19*N each, canonical FP64) are f^n and g^n when
 * pending == 0, or the recorded post-collision fields of step n-1 (as written
 * by lb_step_record) when pending != 0, in which case f^n_i(s) = f_i(s - c_i).
 * phi_n[N] = sum_i g^n_i (as lb_step_record writes it for step n), or NULL to
 * have it computed from g.
 * lf_next, lg_next = dL/df^{n+1}, dL/dg^{n+1}; lf_n, lg_n receive dL/df^n and
 * dL/dg^n (must not alias the inputs or each other).  grads (device
 * doubles) is INCREMENTED by dL/d(1/tau_f), dL/d(1/tau_g) and dL/dkappa of
 * this step (tau_g = mobility/gamma + 1/2); then, for LB_TRT, by
 * dL/d(1/tau_minus) (tau_f being the time of the even part of f - f^eq),
 * and for LB_MRT by dL/d(1/tau) of tau_minus, tau_bulk, tau_ghost_even and
 * tau_ghost_odd (tau_f being the shear time): 3 doubles for LB_BGK, 4 for
 * LB_TRT, 7 for LB_MRT.  With TRT or MRT the symmetric relaxation Omega
 * takes the place of 1/tau_f as in lb_adjoint_step.  Uses the context's parameters;
 * uses the context's spare state buffer and phi buffer as scratch, so calls
 * on one context must not overlap; the lattice state itself is unchanged.
 * Not in the paper (it has no adjoint); the transpose of Section IV's
 * binary step as this library computes it.  LB_ENOTSUP for LB_SINGLE or
 * reduced storage; LB_EINVAL on NULL or aliasing arrays. */
int lb_adjoint_step_binary(lb_ctx* ctx, const double* f, const double* g, const double* phi_n,
                           int pending, const double* lf_next, const double* lg_next,
                           double* lf_n, double* lg_n, double* grads);

/* Reverse of lb_init_equilibrium for LB_BINARY + LB_F64: given rho[N],
 * u[3*N], phi[N] (the initial fields, as passed to lb_init_equilibrium) and
 * lf0, lg0 = dL/df^0, dL/dg^0 (19*N each), writes dphi[N] = dL/dphi,
 * drho[N] = dL/drho, du[3*N] = dL/du and INCREMENTS *dkappa (one device
 * double) by the dependence of the initial state on kappa.  Any collision
 * (the initial state does not relax).  Same scratch rule as
 * lb_adjoint_step_binary.  Not in the paper (transpose of lb_init_equilibrium).
 * LB_ENOTSUP for LB_SINGLE or reduced storage; LB_EINVAL on NULL. */
int lb_adjoint_init_binary(lb_ctx* ctx, const double* rho, const double* u, const double* phi,
                           const double* lf0, const double* lg0, double* dphi, double* drho,
                           double* du, double* dkappa);

/* Reverse sweep over one recorded segment of `length` >= 1 steps, in one
 * call: the same result as `length` calls of the per-step adjoint, for steps
 * n = s0+length-1 down to s0, with the adjoint fields kept on the device
 * between them (the checkpoint/recompute scheme of the adjoint section:
 * the segment is re-run from its checkpoint with lb_step_record, then
 * reversed here).  FP64, same model and collision restrictions as the
 * per-step calls (LB_ENOTSUP otherwise); length < 1 is LB_EINVAL.
 *
 * lb_adjoint_segment (LB_SINGLE, any collision): f0[19*N] = f^{s0} (canonical, not pending);
 * post = the length-1 post-collision fields lb_step_record(length-1) wrote
 * from f^{s0} (19*N each, consecutive; NULL when length == 1).  lam[19*N]
 * holds dL/df^{s0+length} on entry and dL/df^{s0} on return; work[19*N] is
 * scratch.  domega (1, 2 or 5 doubles) is INCREMENTED as by lb_adjoint_step, step by step in
 * the same order, so the result equals the per-step calls bit for bit.
 *
 * lb_adjoint_segment_binary (LB_BINARY): f0, g0 = f^{s0}, g^{s0}; post = the
 * length-1 records of lb_step_record (38*N each: f then g; NULL when
 * length == 1); phi = the length-1 phi fields recorded with them (N each), or
 * NULL to have every step's phi computed.  lf, lg (19*N each) hold
 * dL/df, dL/dg at step s0+length on entry and at s0 on return; work[38*N]
 * is scratch.  grads (3, 4 or 7 device doubles) is INCREMENTED as by
 * lb_adjoint_step_binary.  Between steps lambda_g is kept as a pair
 * (P, b), P_j(x) = lambda_g^{n+1}_j(x + c_j) and b = dL/dphi^n, from which
 * lambda_g^n = (1 - 1/tau_g) P + b; this moves 136 fewer bytes a site per
 * step than the per-step call, and agrees with it to rounding.
 *
 * No argument array may alias another (LB_EINVAL where detected).  Both use
 * the context's spare state buffer and phi buffer as scratch (calls on one
 * context must not overlap; the lattice state is unchanged).  With
 * lb_profile on, every kernel of the sweep is timed as LB_K_ADJOINT, one
 * record per step's local kernel (single: the k_adjoint launch).
 * Not in the paper (it has no adjoint). */
int lb_adjoint_segment(lb_ctx* ctx, const double* f0, const double* post, int32_t length, double* lam,
                       double* work, double* domega);
int lb_adjoint_segment_binary(lb_ctx* ctx, const double* f0, const double* g0, const double* post,
                              const double* phi, int32_t length, double* lf, double* lg, double* work,
                              double* grads);

/* Masked transfer (the masked host/target copies of Section III-B, which pack
 * the selected sites on the device so that only they cross to the host).
 * lb_mask_index compacts mask[N] (device uint8, nonzero = site included) into
 * index[0 .. *count) (device int32, capacity N): the included sites in
 * increasing site order; *count is one device int64.  Deterministic.
 * lb_get_sites gathers the current state at index[0 .. m) into f_packed and
 * g_packed (device, storage dtype, direction-major: element (i, t) at
 * i*m + t; g_packed only for LB_BINARY, else NULL); lb_set_sites writes them
 * back into the state (sites outside [0, N) are skipped; listing a site twice
 * leaves one of the two values).  m = 0 is a no-op; m < 0 or m > N is
 * LB_EINVAL.  Paper: Section III-B (copyFromTargetMasked /
 * copyToTargetMasked: a boolean structure of size N selects the sites, a
 * kernel packs them into a scratch structure on the target; the host-side
 * unpack loop is the caller's).  lb_mask_index keeps its block counts in the
 * context's partial-sum area. */
int lb_mask_index(lb_ctx* ctx, const uint8_t* mask, int32_t* index, int64_t* count);
int lb_get_sites(lb_ctx* ctx, const int32_t* index, int64_t m, void* f_packed, void* g_packed);
int lb_set_sites(lb_ctx* ctx, const int32_t* index, int64_t m, const void* f_packed, const void* g_packed);

/* Per-kernel timing with HIP events on the context's stream.
 * lb_profile(ctx, 1) starts recording an event pair around every kernel
 * launch (and clears earlier records); lb_profile(ctx, 0) stops.  The events
 * are created without the system-scope fence (hipEventDisableSystemFence):
 * they time the work between them but do not publish its memory to the host.
 * lb_kernel_times waits for the recorded events and returns, for kernel
 * class `kind`, the summed duration in milliseconds and the launch count.
 * Not in the paper (measurement; its Section IV reports whole-run times). */
#define LB_K_COLLIDE  0   /* collide / fused pull-stream + collide */
#define LB_K_PHI      1   /* order-parameter kernel (binary) */
#define LB_K_STREAM   2   /* stand-alone propagation */
#define LB_K_ADJOINT  3   /* adjoint step (binary: its phi, local and stencil kernels) */
#define LB_K_OTHER    4   /* init, moments, sums, copies */
int lb_profile(lb_ctx* ctx, int enable);
/* As lb_profile, but only launches of the kernel classes whose bits are set
 * in `kinds` (bit k = 1 << LB_K_...) get an event pair; the others run
 * unbracketed, so a measurement of one class perturbs the rest less.
 * kinds = 0 stops; bits above LB_K_OTHER are LB_EINVAL. */
int lb_profile_mask(lb_ctx* ctx, unsigned kinds);
int lb_kernel_times(lb_ctx* ctx, int kind, double* total_ms, int64_t* launches);

/* Destroy a context (waits for its stream).  NULL is allowed (LB_OK).
 * The workspace is not freed: it belongs to the caller.  Paper: Section
 * III-B (targetFree), except that the memory is the caller's. */
int lb_destroy(lb_ctx* ctx);

/* Streaming copy: dst[0 .. bytes) = src[0 .. bytes), device pointers, both
 * 16-byte aligned, bytes a multiple of 16, the two ranges disjoint; queued
 * on `stream` (a hipStream_t, NULL = the null stream).  Every byte is read
 * once and written once with 16-byte accesses (nontemporal stores, as in the
 * step kernels): the HBM rate of a plain copy on this memory system, which
 * bounds the step kernels in practice, and the reference kernel that turns
 * the HBM byte counters of a profiler into bytes.  Needs no context.
 * bytes == 0 is a no-op; LB_EINVAL on NULL, misalignment, overlap or a
 * grid beyond 2^31 - 1 blocks.  Not in the paper (measurement). */
int lb_stream_copy(void* dst, const void* src, size_t bytes, void* stream);

/* Allocation-free variant of lb_conserved_sums, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): no context and no workspace.  out[5]
 * (device, FP64) = (sum rho, sum j_x, sum j_y, sum j_z, sum phi) of the
 * state f (and g for LB_BINARY; NULL for LB_SINGLE) given in the canonical
 * layout and storage dtype of *p (as lb_get_state writes it: 19*N values
 * each, deviations for LB_F32 / LB_F16 with p->rho0, p->phi0), all device
 * pointers of the current device, queued on `stream`.  Only p's extents,
 * model, storage, rho0 and phi0 are read (the rest must still be valid).
 * The same kernels and summation order as lb_conserved_sums on a context
 * holding that state unpropagated, so the two give identical bits.
 * Partial sums go to a fixed array of the library on each device, of
 * LB_NOALLOC_MAX_BLOCKS blocks of 64 bytes (16 MiB, held by each device the
 * library runs on until the process ends; every value read was written by
 * the same call, so nothing needs clearing): lattices with
 * ceil(nx/64) * ceil(ny/4) * nz > LB_NOALLOC_MAX_BLOCKS (a cube above
 * 384^3, say) give LB_ERANGE.  Calls that overlap on one device (several
 * streams, several threads) share that array and race; serialise them.
 * Allocates nothing: no hipMalloc, no workspace.  LB_EINVAL on NULL or bad
 * parameters; LB_EDEVICE if the device array cannot be located. */
#define LB_NOALLOC_MAX_BLOCKS 262144
int lb_conserved_sums_noalloc(const lb_params* p, const void* f, const void* g, double* out, void* stream);

/* Static description of a status code.  Not in the paper. */
const char* lb_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* LB_H */
