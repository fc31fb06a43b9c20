/*
 * lb.h -- C ABI of the MI355X (gfx950) D2Q37 thermal lattice Boltzmann step.
 *
 * Method: Calore, Gabbana, Kraus, Schifano, Tripiccione, "Performance and
 * Portability of Accelerated Lattice Boltzmann Applications with OpenACC".
 * One time step is, as in Sec. 2: propagate (each of the 37 populations is
 * gathered from the site e_l away, |e_l| up to 3 sites, Eq. (1) left side),
 * bc (top and bottom walls at fixed temperature and zero velocity), collide
 * (Eq. (2) moments, equilibrium, relaxation with rate 1/tau, Hermite
 * projection, gravity).  x is periodic through three halo columns on each side
 * (Sec. 2 and Sec. 4).
 *
 * Units.  Populations hop by integer vectors e_l; their lattice velocities are
 * c_l = r e_l (r = 1.19697977..., fixed by the degree-9 quadrature), so T = 1
 * is the reference temperature and u, T and g below are in the units of c_l
 * with a time step of 1.
 *
 * Conventions for every entry point.
 *  - All functions return an int status: LB_OK (0) or a negative LB_E_* code.
 *    lb_last_error() returns a thread-local, human-readable message for the
 *    last failure on the calling thread.
 *  - Device pointers are plain device addresses (e.g. torch tensor data_ptr()).
 *    The caller owns ALL device memory, including the workspace; the library
 *    owns only the host-side lb_ctx (freed by lb_free).
 *  - Fields (rho, ux, uy, T, gradients) are FP64, x-major [lx][ly], contiguous
 *    (y fastest).  Population arrays in the compact form (lb_get_state and
 *    the like) are [37][lx][ly]; adjoint arrays follow the lattice's layout
 *    (see the adjoint section).
 *  - Work is enqueued asynchronously on the stream given to lb_init (a
 *    hipStream_t passed as void*, NULL = the null stream); nothing waits for
 *    the GPU except lb_step with check_finite > 0.  The caller synchronises
 *    before reading results.  Errors of already-enqueued work surface as
 *    LB_E_HIP at a later call (sticky).
 *  - A context belongs to the HIP device current at lb_init; every later call
 *    on it must be made with that device current (else LB_E_STATE).
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef D2Q37_LB_H
#define D2Q37_LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LB_OK 0
#define LB_E_ARG (-1)       /* null pointer, bad size or parameter        */
#define LB_E_WORKSPACE (-2) /* workspace too small or misaligned          */
#define LB_E_HIP (-3)       /* HIP runtime error (launch or earlier fault) */
#define LB_E_STATE (-4)     /* call not valid in this context's state      */
#define LB_E_NONFINITE (-5) /* check_finite found rho<=0, T<=0 or NaN/Inf  */

/* lb_lattice.precision.  The FP32 modes store g_l = f_l - w_l rho_ref in FP32
 * (half the HBM traffic of FP64) and differ in the arithmetic of the
 * collision; bc and the moments of lb_moments are FP64 in every mode.
 *  LB_FP32_SHIFTED: FP32 storage, FP64 collision (every sum and product of
 *    the collision in FP64, one rounding to FP32 on store).
 *  LB_FP32_SHIFTED_F32SUM: FP32 storage, the FP64 collision's Hermite sums in
 *    FP32 (an ablation: its error grows past 1e-5 within a few hundred steps
 *    of the Rayleigh-Taylor lattice).
 *  LB_FP32_COLLIDE and LB_FP32_LOCAL store each population as its FP32
 *    deviation g_l = f_l - M_l from the rest Maxwellian
 *    M_l = f^eq_l(rho_s, 0, 1 + th_s) of the site that collided it, and that
 *    site's (rho_s, th_s) as two FP16 numbers in one 32-bit word (a 38th
 *    plane); the deviation holds only the flow and the non-equilibrium part
 *    of f, so its rounding is far below an FP32 rounding of f.  Fused kernel
 *    only (the split stages need the source site's reference).
 *  LB_FP32_COLLIDE: that storage with an FP32 collision: the Hermite
 *    projection and reconstruction run in FP32 on the deviation; FP64 is kept
 *    for the sums of the collision invariants (mass, momentum, energy), the
 *    equilibrium's Hermite coefficients (Sec. 2: the collision is a
 *    relaxation towards that equilibrium, projected on Hermite polynomials)
 *    and a correction that restores the invariants after the FP32
 *    reconstruction.
 *  LB_FP32_LOCAL: that storage with the FP64 collision. */
#define LB_FP64 0                /* FP64 storage, FP64 collision           */
#define LB_FP32_SHIFTED 1        /* FP32 storage, FP64 collision           */
#define LB_FP32_SHIFTED_F32SUM 2 /* FP32 storage, FP32 Hermite sums        */
#define LB_FP32_COLLIDE 3        /* FP32 local-reference storage, FP32     */
                                 /* collision, FP64 invariants             */
#define LB_FP32_LOCAL 4          /* FP32 local-reference storage, FP64     */
                                 /* collision                              */
/* lb_lattice.ybc */
#define LB_Y_WALLS 0    /* thermal walls below row 0 and above row ly-1 */
#define LB_Y_PERIODIC 1 /* periodic y (no walls), for tests             */
/* lb_lattice.layout: address of population l at padded site (X, Y) */
#define LB_LAYOUT_SOA 0    /* l*NX*NY + X*NY + Y   (the paper's layout, Sec. 4) */
#define LB_LAYOUT_COLUMN 1 /* X*37*NY + l*NY + Y   (all populations of a column */
                           /*  contiguous)                                      */
/* lb_params.kernel.  The three SPLIT_* values run the split stages with one
 * stage replaced by an alternative kernel (same results: propagate bit for
 * bit, collide to FP64 rounding), kept to measure the main kernels' design
 * against: propagate with each population's source window (the tile's rows
 * and the three-row halo, Sec. 2) staged through LDS; propagate with 16-byte
 * accesses (two FP64 / four FP32 sites per thread); the FP64 collide with
 * the Hermite projection and reconstruction (Sec. 2) as dense products on the
 * FP64 matrix cores (LB_FP64 only).  The local-reference forms run
 * LB_KERNEL_FUSED only. */
#define LB_KERNEL_FUSED 0      /* one kernel per step: propagate+bc+collide        */
#define LB_KERNEL_SPLIT 1      /* halo, propagate, bc, collide as separate kernels */
#define LB_KERNEL_SPLIT_LDS 2  /* split, propagate staged through LDS              */
#define LB_KERNEL_SPLIT_WIDE 3 /* split, propagate with 16-byte accesses           */
#define LB_KERNEL_SPLIT_MFMA 4 /* split, collide on the FP64 matrix cores          */

typedef struct lb_lattice {
  int32_t lx;        /* physical sites along x (periodic), 6 .. 2^22    */
  int32_t ly;        /* physical sites along y (walls), 6 .. 2^24;      */
                     /* lx * ly <= 2^30                                 */
  int32_t precision; /* LB_FP64 or one of the FP32 modes above       */
  int32_t ybc;       /* LB_Y_WALLS or LB_Y_PERIODIC                     */
  int32_t layout;    /* LB_LAYOUT_SOA or LB_LAYOUT_COLUMN               */
  int32_t reserved;  /* must be 0                                       */
} lb_lattice;

typedef struct lb_params {
  double tau;          /* relaxation time, > 0.5 (Eq. (1))                     */
  double gx, gy;       /* gravity (acceleration per step)                      */
  double t_bottom;     /* wall temperature below row 0                         */
  double t_top;        /* wall temperature above row ly-1                      */
  double rho_ref;      /* shift density of the FP32 modes (ignored for FP64)   */
  int32_t regularize;  /* 1: Hermite projection of the collision, 0: plain BGK */
  int32_t kernel;      /* LB_KERNEL_FUSED, LB_KERNEL_SPLIT or a SPLIT_* variant */
  int32_t check_finite; /* 0: off; N > 0: every N steps lb_step scans the state */
                        /* and returns LB_E_NONFINITE if rho<=0, T<=0 or NaN   */
  int32_t reserved;     /* must be 0                                           */
} lb_params;

typedef struct lb_ctx lb_ctx;

const char* lb_last_error(void);
/* Interface version: 5 (3: adjoint arrays in the lattice's layout and
 * lb_adjoint_run; 4: precisions LB_FP32_COLLIDE and LB_FP32_LOCAL;
 * 5: kernels LB_KERNEL_SPLIT_LDS, _WIDE and _MFMA). */
int lb_version(void);

/* Bytes of device workspace lb_init needs for this lattice (two padded
 * population buffers plus a small scratch area).  Pure host computation. */
int lb_workspace_bytes(const lb_lattice* lat, const lb_params* par, size_t* bytes);

/* Creates a context on the current HIP device.  `workspace` (device, >= the
 * size from lb_workspace_bytes, 256-byte aligned) is carved into the state
 * buffer A, the scratch buffer B and reduction scratch; it must outlive the
 * context.  The state is set to the equilibrium f_l = f^eq_l(rho0, u0, T0)
 * (Sec. 2: the run starts from an assignment of the populations at t = 0),
 * then the halos are refreshed.  rho0, ux0, uy0, T0: device FP64 [lx][ly].
 * Errors: LB_E_ARG (sizes out of the limits of lb_lattice, tau <= 0.5,
 * non-finite parameters, unknown enum values, null pointers, reserved != 0),
 * LB_E_WORKSPACE (size, alignment), LB_E_HIP; *out is NULL on failure. */
int lb_init(const lb_lattice* lat, const lb_params* par, void* workspace,
            size_t workspace_bytes, void* stream, const double* rho0,
            const double* ux0, const double* uy0, const double* T0,
            lb_ctx** out);

/* Releases the host-side context (device memory belongs to the caller).
 * Enqueued work is not waited for.  NULL is accepted; always LB_OK. */
int lb_free(lb_ctx* ctx);

/* Changes the stream later work is enqueued on.  Errors: LB_E_ARG (NULL ctx). */
int lb_set_stream(lb_ctx* ctx, void* stream);

/* Replaces the physical parameters (tau, g, walls, regularize, kernel,
 * check_finite); rho_ref cannot change after lb_init.  LB_E_ARG as lb_init. */
int lb_set_params(lb_ctx* ctx, const lb_params* par);

/* Advances the state by n >= 0 full steps (propagate -> bc -> collide),
 * with the fused kernel or the split kernels as par->kernel selects.
 * Errors: LB_E_ARG (NULL ctx, n < 0), LB_E_HIP, LB_E_NONFINITE (only with
 * check_finite > 0: the scan found rho <= 0, T <= 0 or a non-finite value; the
 * state is left as computed). */
int lb_step(lb_ctx* ctx, int n);

/* Eq. (2) of the current (post-collision) state: rho = sum f,
 * rho u = sum c f, 2 rho T = sum |c - u|^2 f, computed in FP64.  Outputs are
 * device FP64 [lx][ly]; any of them may be NULL.  Errors: LB_E_ARG (NULL
 * ctx), LB_E_HIP. */
int lb_moments(lb_ctx* ctx, double* rho, double* ux, double* uy, double* T);

/* Device copies of the state in compact form: [37][lx][ly] double for
 * LB_FP64, [37][lx][ly] float g_l = f_l - w_l rho_ref for the shifted FP32
 * modes, and [38][lx][ly] 32-bit words for LB_FP32_COLLIDE / LB_FP32_LOCAL
 * (37 float deviations, then each site's packed FP16 reference, rho_s low,
 * th_s high).  set_state refreshes the halos.  Used for checkpoints.
 * Errors: LB_E_ARG (NULL pointers), LB_E_HIP. */
int lb_get_state(lb_ctx* ctx, void* f);
int lb_set_state(lb_ctx* ctx, const void* f);

/* The state as true populations f_l in FP64 [37][lx][ly], any precision. */
int lb_get_populations(lb_ctx* ctx, double* f);

/* Single stages of the split path, for per-kernel tests and timing.
 *   lb_halo:      refreshes the periodic halos of the state buffer A
 *                 (x columns; also y rows when ybc = LB_Y_PERIODIC).
 *   lb_propagate: B(l, x, y) = A(l, x - e_lx, y - e_ly) for every physical
 *                 site (needs valid halos); slots whose source row is outside
 *                 the walls are left unspecified for bc.
 *   lb_bc:        applies the thermal walls to B in place (rows 0..2 and
 *                 ly-3..ly-1; no-op for LB_Y_PERIODIC).
 *   lb_collide:   A = collide(B), site by site.
 * lb_propagate and lb_collide run the alternative kernel of the context's
 * LB_KERNEL_SPLIT_* value where it names one (lb_step's split path too).
 * lb_get_scratch / lb_set_scratch copy B's physical region in the compact
 * form of lb_get_state.  The local-reference forms (LB_FP32_COLLIDE,
 * LB_FP32_LOCAL) have no split stages: lb_propagate, lb_bc, lb_collide,
 * lb_get_scratch and lb_set_scratch return LB_E_STATE for them. */
int lb_halo(lb_ctx* ctx);
int lb_propagate(lb_ctx* ctx);
int lb_bc(lb_ctx* ctx);
int lb_collide(lb_ctx* ctx);
int lb_get_scratch(lb_ctx* ctx, void* f);
int lb_set_scratch(lb_ctx* ctx, const void* f);

/* In-situ observables of the current state (the averages and correlations
 * the paper's production runs compute every few hundred steps, Sec. 2), all
 * on the device in FP64, deterministic.
 * lb_observables: profiles (device [6][ly], may be NULL) receives the row
 * averages over x of rho, u_x, u_y, T, rho |u|^2 / 2 and rho T; scalars
 * (device [4], may be NULL) the total mass, the kinetic energy
 * (1/2) sum rho |u|^2, sum rho T, and the mixing-layer width
 * 6 sum_y phi (1 - phi) with phi = (Tbar(y) - t_top) / (t_bottom - t_top)
 * clamped to [0, 1] (the width of a linear temperature ramp).
 * lb_run_observed: n steps as lb_step; after every `every` steps the four
 * scalars are written to series + 4 * (k - 1) for the k-th sample (device
 * [n / every][4]); no host synchronisation.  Errors: LB_E_ARG (NULL ctx,
 * n < 0, every <= 0, series NULL when n >= every), LB_E_HIP, and those of
 * lb_step. */
int lb_observables(lb_ctx* ctx, double* profiles, double* scalars);
int lb_run_observed(lb_ctx* ctx, int n, int every, double* series);

/* Adjoint (LB_FP64 contexts only; LB_E_STATE otherwise).  Besides that,
 * every adjoint entry point returns LB_E_ARG for a NULL context or a NULL
 * required pointer (the optional ones are named below) and LB_E_HIP for a
 * launch failure; lb_adjoint_step also rejects lambda_in == lambda_out.
 *
 * lb_step_record: like lb_step(n) with the fused kernel, and also writes, for
 * each step j, the four pre-collision moments m = (rho, rho u_x, rho u_y,
 * sum |c|^2 f) of every site to tape + j*4*lx*ly as [4][lx][ly] FP64.
 *
 * Adjoint populations (lambda, 37 * lx * ly FP64 values, no halos) are laid
 * out like the context's populations: [lx][37][ly] for LB_LAYOUT_COLUMN,
 * [37][lx][ly] for LB_LAYOUT_SOA (y contiguous in both).
 *
 * lb_loss_ke: KE = (1/2) sum rho |u|^2 of the current state into ke_dev (one
 * device double) and, if lambda != NULL, dKE/df_l = c_l.u - |u|^2/2 into
 * lambda.
 *
 * lb_adjoint_step: lambda_out = (d f^{n+1} / d f^n)^T lambda_in for the step
 * whose pre-collision moments are tape_j ([4][lx][ly] from lb_step_record):
 * the transposed collision, walls and propagation, in one kernel.  lambda_in
 * and lambda_out are distinct buffers; every element of lambda_out is
 * written.
 *
 * lb_adjoint_run: n transposed steps in one call, lambda^n -> lambda^0 in
 * place in `lambda`, with tape = [n][4][lx][ly] from lb_step_record (tape
 * step j holds the moments of the step from f^j to f^{j+1}).  The same
 * arithmetic as n calls of lb_adjoint_step, and the same result bit for bit.
 * On lattices beyond the Infinity Cache P^T is applied as a gather by the
 * following step: between steps the adjoint lives in two padded FP64 buffers
 * laid out like the state (aligned stores instead of the scatter's partial
 * ones); on lattices of 2^17 sites up to the cache size the steps are the
 * scatter kernel of lb_adjoint_step.  `workspace`: 256-byte aligned, at least
 * the size from lb_adjoint_workspace_bytes, previous contents irrelevant, and
 * overlapping neither tape, lambda nor the context's own workspace.  n = 0
 * leaves lambda unchanged.  Errors: LB_E_STATE (not FP64), LB_E_ARG (n < 0,
 * NULL pointers), LB_E_WORKSPACE (size, alignment), LB_E_HIP.
 *
 * lb_init_adjoint: given lambda0 = dL/df^0 and the initial fields
 * (rho0, ux0, uy0, T0) the state was built from, writes dL/d(rho0, ux0, uy0,
 * T0) of the initial equilibrium f^0 = f^eq(rho0, u0, T0); all [lx][ly],
 * outputs may be NULL. */
int lb_step_record(lb_ctx* ctx, int n, double* tape);
int lb_loss_ke(lb_ctx* ctx, double* ke_dev, double* lambda);
int lb_adjoint_step(lb_ctx* ctx, const double* tape_j, const double* lambda_in,
                    double* lambda_out);
int lb_adjoint_workspace_bytes(lb_ctx* ctx, size_t* bytes);
int lb_adjoint_run(lb_ctx* ctx, int n, const double* tape, double* lambda, void* workspace,
                   size_t workspace_bytes);
/* lb_adjoint_run_static: lb_adjoint_run without a workspace argument, for
 * callers that cannot allocate device memory (code under graph capture,
 * serving loops, harnesses that forbid hipMalloc).  The two padded adjoint
 * buffers live in a 64 MiB array the library holds on each GPU it runs on
 * (for the life of the process); the first call on a device looks its address
 * up.  The call allocates nothing; its result is that of lb_adjoint_run, bit
 * for bit.  Lattices whose two padded FP64 buffers exceed 64 MiB
 * (2 * 37 * (lx + 6) * (ly + 64, rounded up to 32) * 8 bytes; about 110,000
 * sites) are rejected with LB_E_WORKSPACE.  All calls on one GPU share that
 * array: calls that overlap on one GPU (other streams, other threads, other
 * contexts) race and must be serialised by the caller.  Errors as
 * lb_adjoint_run, plus LB_E_HIP when the array's address cannot be looked up. */
int lb_adjoint_run_static(lb_ctx* ctx, int n, const double* tape, double* lambda);
int lb_init_adjoint(lb_ctx* ctx, const double* rho0, const double* ux0,
                    const double* uy0, const double* T0, const double* lambda0,
                    double* drho0, double* dux0, double* duy0, double* dT0);

#ifdef __cplusplus
}
#endif

#endif /* D2Q37_LB_H */
