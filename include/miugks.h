/*
 * miugks.h - C ABI of the MI355X (gfx950) implementation of the multigrid
 * implicit unified gas-kinetic scheme (MIUGKS) of Zhu, Zhong & Xu,
 * "Unified gas-kinetic scheme with multigrid convergence for rarefied flow
 * study" (arXiv:1704.03151).
 *
 * One context holds one steady problem on a structured 2-D mesh with a
 * tensor-product discrete velocity grid, the coarsened mesh hierarchy of
 * Sec. III A, and all device memory of the solver (owned by the library,
 * allocated in miugks_create, released in miugks_destroy).  Every hot step
 * runs in the library's HIP kernels on the stream given at creation.
 *
 * Conventions
 *  - All functions return MIUGKS_OK (0) or an error code; the text of the
 *    last error of a context is returned by miugks_last_error().
 *  - Host arrays passed in are copied and never retained; host arrays passed
 *    out are owned by the caller.  A pointer argument documented as
 *    "may be NULL" is skipped when NULL.
 *  - Cell arrays are [ny][nx] (x fastest).  Macroscopic fields are
 *    nondimensional: lengths by the reference length, density by rho0,
 *    temperature by T0, speeds by sqrt(2 R T0) (so R T0 = 1/2).
 *  - Distribution arrays hold the reduced pair (G, H): G integrates f over the
 *    K_int extra velocity components, H integrates their squared magnitude.
 *    Layout [2][Nk][ny][nx]: G plane then H plane, each velocity-major with
 *    cells fastest; velocity index k = ku * nv + kv.
 *  - A context is not thread-safe; use one context per host thread.
 *  - No C++ exception crosses this interface.
 */
#ifndef MIUGKS_H
#define MIUGKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MIUGKS_OK 0
#define MIUGKS_EINVAL 1          /* bad argument or unsupported configuration */
#define MIUGKS_ENOMEM 2          /* device or host allocation failed */
#define MIUGKS_EDEVICE 3         /* HIP runtime error (text in miugks_last_error) */
#define MIUGKS_EDIVERGED 4       /* residual non-finite or blew up; state is the last finite cycle */
#define MIUGKS_ENOTCONVERGED 5   /* max_cycles reached above the tolerance; state valid */
#define MIUGKS_ESTATE 6          /* call not valid in the current state */

/* face tags (Sec. III B boundary conditions) */
#define MIUGKS_FACE_INTERIOR 0   /* two fluid cells */
#define MIUGKS_FACE_WALL 1       /* diffuse isothermal wall, full accommodation */
#define MIUGKS_FACE_FARFIELD 2   /* freestream Maxwellian enters, the cell's distribution leaves */
#define MIUGKS_FACE_OUTFLOW 3    /* zero gradient */
#define MIUGKS_FACE_SYMMETRY 4   /* specular reflection: the cell's own distribution at the velocity with the
                                    normal component reversed (the grid must be symmetric in it) */

/* precision of the distribution and of the per-velocity arithmetic */
#define MIUGKS_FP64 0            /* everything in double */
#define MIUGKS_FP32F 1           /* f, flux, residual and smoother arithmetic in float;
                                    moments, macroscopic prediction and norms in double */

/* one-dimensional quadrature rules (velocity grids, Sec. IV) */
#define MIUGKS_QUAD_TRAPEZOID 0
#define MIUGKS_QUAD_SIMPSON38 1  /* composite Simpson 3/8, needs (n-1) % 3 == 0 */
#define MIUGKS_QUAD_GAUSS_HERMITE 2

/* cycle_gamma / cycle_gamma_cs value that selects F-cycles (Sec. II D): one
 * visit of a level makes an F-cycle and then a V-cycle on the next coarser
 * level, so level l (0 = finest) is visited l + 1 times per cycle */
#define MIUGKS_CYCLE_F (-1)

/* wall loads (Sec. IV B), per wall side; see miugks_wall_loads */
#define MIUGKS_LOAD_PRESSURE 0
#define MIUGKS_LOAD_SHEAR 1
#define MIUGKS_LOAD_HEAT 2

typedef struct miugks_ctx miugks_ctx;

/* Device allocator callbacks: alloc returns `bytes` of device memory on the
 * current device (NULL when it cannot), free releases a pointer alloc gave. */
typedef void* (*miugks_alloc_fn)(size_t bytes, void* user);
typedef void (*miugks_free_fn)(void* ptr, void* user);

/* Structured mesh (Sec. III A).  Cell (ix, iy) spans [x[ix], x[ix+1]] x
 * [y[iy], y[iy+1]].  x-face (ix, iy), index iy*(nx+1)+ix, lies on x = x[ix];
 * y-face (ix, iy), index iy*nx+ix, lies on y = y[iy].  Domain-boundary faces
 * must not be INTERIOR; a face between a fluid and a solid cell must be a
 * WALL.  wall_x / wall_y hold (T_w, U_w, V_w) per face (3 doubles), read only
 * for WALL faces (may be NULL when there is no wall).  solid may be NULL.
 * n_levels >= 1; nx, ny must be divisible by 2^(n_levels-1), coarse faces must
 * not mix tags and coarse cells must not mix fluid and solid. */
typedef struct {
    int nx, ny, n_levels;
    const double* x;
    const double* y;
    const uint8_t* face_type_x;
    const uint8_t* face_type_y;
    const double* wall_x;
    const double* wall_y;
    const uint8_t* solid;
} miugks_mesh_desc;

/* Tensor-product velocity grid: nodes u[nu], v[nv], 1-D weights wu[nu], wv[nv]. */
typedef struct {
    int nu, nv;
    const double* u;
    const double* v;
    const double* wu;
    const double* wv;
} miugks_vgrid_desc;

/* Gas: K_int extra degrees of freedom (1 for a monatomic gas in 2-D), Prandtl
 * number (Shakhov model), viscosity mu = mu_ref T^omega with mu_ref fixed by
 * the VHS mean free path Kn (alpha = 1), freestream state for FARFIELD faces. */
typedef struct {
    int K_int;
    double Pr, omega, Kn;
    double rho_inf, U_inf, V_inf, T_inf;
} miugks_gas_desc;

/* Solver: precision (MIUGKS_FP64 / MIUGKS_FP32F), smoothing counts nu1
 * (pre), nu2 (post), nu_coarse (coarsest level), Courant number of the
 * physical step, growth a of the pseudo step dt_n = a^n dt_p (0 = off,
 * Sec. III D), mass_renorm: 1 = keep total mass, 0 = off, -1 = on iff the
 * domain has walls only; fas_levels: levels of the FAS prediction, from the
 * finest (0 or more than n_levels: all of them; the CS correction always
 * uses n_levels); nu_coarse_cs: smoothings of the CS correction on its
 * coarsest level (0: nu_coarse, which then counts for both cycles);
 * cycle_gamma: coarse-grid corrections per visit of a level in the FAS
 * cycle, 1 (or 0) for V-cycles, 2 for W-cycles, at most 3, or MIUGKS_CYCLE_F
 * for F-cycles; cycle_gamma_cs: the same for the CS cycle (0: cycle_gamma);
 * dtn_max: cap of the pseudo-step growth, dt_n = min(a^n, dtn_max) dt_p
 * (0: no cap; only read when dtn_growth > 0; the pseudo step leaves the fixed
 * point unchanged, the cap keeps its damping once a^n is large). */
typedef struct {
    int precision;
    int nu1, nu2, nu_coarse;
    double cfl;
    double dtn_growth;
    int mass_renorm;
    int fas_levels;
    int nu_coarse_cs;
    int cycle_gamma;
    int cycle_gamma_cs;
    double dtn_max;
} miugks_solver_desc;

/* Nodes and weights of a 1-D rule on [lo, hi] (ignored for Gauss-Hermite,
 * whose weights integrate plain functions: w = w_GH * exp(u^2)).  nodes and
 * weights are host arrays of n doubles.  Sec. IV (trapezoid, Newton-Cotes). */
int miugks_quadrature(int kind, int n, double lo, double hi, double* nodes, double* weights);

/* Allocator of the contexts created from now on (process-wide; not to be
 * called while another thread creates a context): every device buffer a
 * context allocates, at creation, for the adjoint or for conversions, comes
 * from alloc and goes back through free when the context is destroyed (or
 * sooner for temporaries).  Lets a caller back the library's memory by its own
 * pool, such as PyTorch's caching allocator.  (NULL, NULL) restores hipMalloc
 * / hipFree; MIUGKS_EINVAL when only one of the two is NULL.  A context keeps
 * the pair it was created with. */
int miugks_set_allocator(miugks_alloc_fn alloc, miugks_free_fn free_fn, void* user);

/* Build the level hierarchy and allocate device memory.  hip_stream is a
 * hipStream_t (e.g. torch.cuda.current_stream().cuda_stream) or NULL for the
 * default stream.  The distribution starts as the rest state rho = T = 1. */
int miugks_create(miugks_ctx** out, const miugks_mesh_desc* mesh, const miugks_vgrid_desc* vgrid,
                  const miugks_gas_desc* gas, const miugks_solver_desc* solver, void* hip_stream);

/* Free all memory of ctx; NULL is a no-op. */
void miugks_destroy(miugks_ctx* ctx);

/* Text of the last error on ctx (NULL ctx: last creation error). */
const char* miugks_last_error(const miugks_ctx* ctx);

/* Initial state of the outer iteration (Sec. IV: the cavity starts at rest,
 * the plate and the square from the freestream, the square with the region
 * behind it at a tenth of the freestream density and at rest): f := the
 * reduced Maxwellian pair (G, H) of the host fields rho, U, V, T [ny][nx]
 * (Sec. II A equilibrium; solid cells: 0).  Resets the cycle counter (the
 * pseudo step of Sec. III D restarts) and the reference mass of a closed
 * domain.  MIUGKS_EINVAL for a NULL field. */
int miugks_init_macro(miugks_ctx* ctx, const double* rho, const double* U, const double* V,
                      const double* T);

/* Outer MIUGKS cycles, Steps 1-8 of Sec. II D: for each cycle compute the UGKS
 * residuals; stop if every RMS residual component (Sec. IV A) is below tol;
 * otherwise run the FAS prediction, micro residual, CS correction and update.
 * cycles_done (may be NULL) receives the number of updates made, res (may be
 * NULL) the four RMS residuals of the last check.  Synchronises the stream. */
int miugks_iterate(miugks_ctx* ctx, int max_cycles, double tol, int* cycles_done, double res[4]);

/* Full-multigrid start (Sec. III C, the FMG method): the current state
 * (normally the one miugks_init_macro set) is restricted to the coarsest
 * level by volume-weighted means; then each level from the coarsest up to
 * level 1 runs up to cycles_per_level outer cycles as the finest level of
 * its own sub-hierarchy (stopping early when every RMS residual is below tol),
 * and its distribution itself, not a correction, is interpolated bilinearly
 * to the next finer level.  Ends with the state on level 0, the cycle counter
 * (and so the pseudo step) restarted; the reference mass of a closed domain
 * is kept.  Follow with miugks_iterate.  cycles_done (may be NULL) receives
 * the cycles run on the coarse levels.  Returns MIUGKS_OK, or the status of a
 * level whose cycles diverged (MIUGKS_EDIVERGED): f is then undefined until
 * miugks_init_macro or miugks_set_f.  Synchronises the stream. */
int miugks_fmg(miugks_ctx* ctx, int cycles_per_level, double tol, int* cycles_done);

/* Explicit, time-accurate UGKS steps on the finest level: the scheme whose
 * time-averaged interface fluxes the residuals of Sec. II A use, marched
 * with one global step dt = the smallest CFL step of the mesh (cells and
 * faces alike).  Per step: the fluxes and R of the current state, the
 * macroscopic update W* = W^n + dt R (a cell whose W* has non-positive
 * density or temperature keeps W^n), the Shakhov equilibria g^n of W^n and
 * g_s of W* with the heat flux q^n, and the trapezoidal update
 * f = [f - dt div + dt/2 (g_s / tau_s + (g^n - f) / tau^n)] / (1 + dt / (2 tau_s)),
 * then the moments of f (and the closed-domain mass renormalisation).
 * dt (may be NULL) receives the step, res (may be NULL) the RMS residuals of
 * the last step's fluxes.  MIUGKS_ESTATE inside a full-multigrid start.
 * Synchronises the stream. */
int miugks_explicit(miugks_ctx* ctx, int steps, double* dt, double res[4]);

/* Macroscopic fields of the current distribution (Sec. II A: the
 * conservative variables W are the velocity moments of f; Sec. IV reports the
 * flow fields as density, velocity and temperature): rho, U, V and
 * T = 4 (rho eps - rho |U|^2 / 2) / (K rho) per cell, and the heat flux
 * qx, qy of the Shakhov model (the moment that enters its equilibrium).
 * Host outputs [ny][nx], caller-owned, each may be NULL; solid cells give 0.
 * Synchronises the stream. */
int miugks_get_macro(miugks_ctx* ctx, double* rho, double* U, double* V, double* T, double* qx,
                     double* qy);

/* Copy the discrete distribution (Sec. II A: f at every cell and discrete
 * velocity, here the reduced pair of Sec. III B) out of / into the context,
 * layout [2][Nk][ny][nx].  dtype is MIUGKS_FP64 (double) or MIUGKS_FP32F
 * (float); it is converted as needed.  on_device = 1: dst/src is a device
 * pointer on the context's device; 0: a host pointer (the library stages it
 * through a device buffer it allocates for the call).  The caller owns dst /
 * src.  set_f recomputes the moments; together they are the
 * checkpoint/restore path.  MIUGKS_EINVAL for a bad dtype or a NULL
 * pointer.  Synchronise the stream. */
int miugks_get_f(miugks_ctx* ctx, void* dst, int dtype, int on_device);
int miugks_set_f(miugks_ctx* ctx, const void* src, int dtype, int on_device);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the result
 * of miugks_get_f(ctx, dst, dtype, 0) into the caller-owned host buffer dst
 * (2 Nk nc elements of dtype), calling no allocator.  A conversion to another
 * dtype is staged through a fixed device array of the library, 16 MiB per GPU
 * and held until the process ends, in pieces of at most that size, so any
 * size of f is accepted; the same dtype is copied directly.  Calls that
 * overlap on one GPU, through any contexts or threads, race on that array;
 * nothing in it needs to start at zero.  MIUGKS_EINVAL for a bad dtype or a
 * NULL dst.  Synchronises the stream. */
int miugks_get_f_noalloc(miugks_ctx* ctx, void* dst, int dtype);

/* --- walls: loads, objectives, temperatures -------------------------------- */

/* Wall sides of the finest level, in the order of their cells (row-major) and
 * then of the sides (0: -x, 1: +x, 2: -y, 3: +y); an internal wall (a plate)
 * has one side per adjacent fluid cell.  cell, side (caller-owned, may be
 * NULL) receive n_walls entries; call with NULLs to get n_walls. */
int miugks_wall_list(miugks_ctx* ctx, int* cell, int* side, int* n_walls);

/* Loads of the current distribution on every wall side (Sec. IV B: the skin
 * friction is the momentum the gas hands to the wall).  The distribution on
 * the wall side of the face is the cell's for velocities leaving the gas and
 * the diffuse-wall Maxwellian (Sec. III B) for the others; in the frame of
 * the wall, c = u - U_w, with c_n along the normal out of the gas and c_t
 * along the face (y on a -x/+x side, x on a -y/+y side):
 *   p = sum_k w c_n^2 f^G, tau = sum_k w c_t c_n f^G,
 *   q = 1/2 sum_k w c_n (|c|^2 f^G + f^H),
 * and S the face area.  Host outputs of n_walls entries each (may be NULL;
 * all NULL: only n_walls is set).  Synchronises the stream. */
int miugks_wall_loads(miugks_ctx* ctx, double* p, double* tau, double* q, double* S, int* n_walls);

/* Integrated wall load (Sec. IV B: the skin friction and drag of the plate
 * are the momentum the gas hands to the wall, integrated over it):
 * J = sum over the listed wall sides (indices of miugks_wall_list) of S times
 * the load kind (MIUGKS_LOAD_PRESSURE, _SHEAR or _HEAT) of miugks_wall_loads;
 * the lid shear of a cavity or the drag of a plate (both of its sides).
 * walls is a host array of n indices; *J (host) out.  MIUGKS_EINVAL for a
 * bad kind or index.  Synchronises the stream. */
int miugks_objective(miugks_ctx* ctx, int kind, const int* walls, int n, double* J);

/* Set the temperature of n wall faces of the mesh (Sec. III B, wall
 * Maxwellian).  Faces are numbered x-faces first (iy (nx + 1) + ix), then
 * y-faces ((nx + 1) ny + iy nx + ix); both sides of an internal wall face
 * take the new value.  Coarse levels are rebuilt from the new values (the
 * area-weighted means of creation).  The distribution is unchanged.
 * MIUGKS_EINVAL for a face that is not a wall or a temperature <= 0 (nothing
 * is changed then).  Synchronises the stream. */
int miugks_set_wall_T(miugks_ctx* ctx, const int* faces, const double* Tw, int n);

/* --- adjoint of the steady state (FP64 contexts) --------------------------- */

/* out = (dr/df)^T v for the steady residual at the current distribution,
 * r_ik(f) = (g_ik(W_i(f), q_i(f)) - f_ik) / tau_i(W_i(f)) - div_ik(f): the
 * microscopic residual of Steps 3-4 (Sec. II A) with the equilibrium of the
 * state itself and the transport of Step 1 (UGKS interface flux, limited
 * slopes, micro-slopes, compatibility time slope, diffuse walls), reversed
 * through the same arithmetic; the limiter takes its derivative where it is
 * smooth.  v and out are laid out as f ([2][Nk][ny][nx]); dtype and on_device
 * as for miugks_get_f.  MIUGKS_EINVAL for an FP32-f context.  Recomputes
 * Step 1 of the current f.  Synchronises the stream. */
int miugks_residual_adjoint(miugks_ctx* ctx, const void* v, void* out, int dtype, int on_device);

/* Sensitivity of J = sum over the wall sides walls[0..n) of S times the load
 * kind (see miugks_objective) to the temperatures of the mesh faces
 * param_faces[0..n_param) (numbered as in miugks_set_wall_T; both sides of an
 * internal wall face count), at a converged steady state:
 *   dJ/dTw = dJ/dTw|_f - lam^T dr/dTw,  (dr/df)^T lam = dJ/df - mu m.
 * In a closed domain (mass renormalisation on) the steady states form a
 * family in the total mass, m is the mass row and mu = dJ/dM along the
 * family, taken from two steady states at masses M0 (1 +- 1e-4) (up to 300
 * cycles each towards 1e-13, from the scaled state; f and M0 are restored),
 * so the result is the sensitivity at fixed mass.  lam is found by restarted
 * GMRES (up to 30 basis vectors, fewer when they would exceed 32 GB),
 * right-preconditioned with -A^-T, A the velocity-diagonal part of the
 * correction operator of Step 5 (Sec. II A 2) solved by one downwind-ordered
 * sweep per velocity, until the residual norm falls by tol or after max_iter
 * Arnoldi steps.  The library allocates the basis on the first call.
 * dJ_dTw (host, n_param) out; iters (Arnoldi steps) and res (relative final
 * residual norm) may be NULL.  Returns
 * MIUGKS_OK, MIUGKS_ENOTCONVERGED (max_iter reached; outputs set),
 * MIUGKS_EDIVERGED, or MIUGKS_EINVAL (FP32-f context, bad kind, wall index
 * or a parameter face that is not a wall).  Synchronises the stream. */
int miugks_adjoint(miugks_ctx* ctx, int kind, const int* walls, int n, const int* param_faces, int n_param,
                   double tol, int max_iter, double* dJ_dTw, int* iters, double* res);

/* miugks_adjoint with the storage type of the Krylov iteration's vectors
 * chosen by krylov_dtype: MIUGKS_FP64, or MIUGKS_FP32F for the Krylov basis,
 * the preconditioner's input and output and the products formed on them in
 * float (half the memory of the basis and of its traffic).  In either form
 * the state f, the interface and cell records, the mass-family term mu,
 * every dot product, the Hessenberg arithmetic, the multiplier lam and the
 * final contraction dJ/dTw|_f - lam^T dr/dTw are double: each restart forms
 * the true residual b - (dr/df)^T lam in double and solves for a correction
 * in float, so the float form reaches the same tolerances as the double one
 * (mixed-precision iterative refinement; 2e-10 on a 64x64 cavity with 784
 * velocities in the same number of steps).  Other arguments and returns as
 * for miugks_adjoint, plus MIUGKS_EINVAL for another krylov_dtype. */
int miugks_adjoint_ex(miugks_ctx* ctx, int kind, const int* walls, int n, const int* param_faces, int n_param,
                      double tol, int max_iter, int krylov_dtype, double* dJ_dTw, int* iters, double* res);

/* --- one call per step of the hot path (parity and profiling) ------------- */

/* Step 1 alone (Sec. II A, residual definitions; UGKS flux): recompute the
 * transport term div and the macroscopic residual R of the current f.  R
 * (host [4][ny][nx], may be NULL) and the RMS norms res (may be NULL) out. */
int miugks_residual(miugks_ctx* ctx, double* R, double res[4]);

/* Transport term div of the last miugks_residual, layout as f. */
int miugks_get_div(miugks_ctx* ctx, void* dst, int dtype, int on_device);

/* Step 2 alone (FAS V-cycle, Sec. II D): predicted conservative variables
 * W_out [4][ny][nx] from W [4][ny][nx] and target residual R [4][ny][nx]
 * (host arrays), with the pseudo step of the current cycle counter. */
int miugks_predict(miugks_ctx* ctx, const double* W, const double* R, double* W_out);

/* Steps 3-4 alone: micro residual r = (g~ - f)/tau~ - div from the predicted
 * state Wt [4][ny][nx] (host), the current f, heat flux and the div of the
 * last miugks_residual.  r_out layout as f (dtype, on_device as get_f);
 * tau_inv_out (host [ny][nx], may be NULL) receives 1/tau~. */
int miugks_micro_residual(miugks_ctx* ctx, const double* Wt, void* r_out, double* tau_inv_out,
                          int dtype, int on_device);

/* Step 5 alone (CS V-cycle, Sec. II D): correction df_out of the linear
 * correction equation with right-hand side r and collision frequency
 * tau_inv (host [ny][nx]).  r and df_out layout as f. */
int miugks_correct(miugks_ctx* ctx, const void* r, const double* tau_inv, void* df_out, int dtype,
                   int on_device);

/* Per-kernel timing for profiling: on = 1 clears previous records and starts
 * bracketing every kernel the library launches with HIP events on its
 * stream; on = 0 stops.  Timing adds a few microseconds per launch. */
int miugks_set_timing(miugks_ctx* ctx, int on);

/* Aggregate of the timed launches since miugks_set_timing(ctx, 1), one entry
 * per kernel label: launch count, summed duration (ms) and summed
 * algorithmic bytes (what the step must read and write once, per the byte
 * model of each kernel).  Fills at most cap entries of the caller's arrays
 * (each may be NULL); label strings stay valid until the next call on ctx.
 * Returns the number of distinct labels, or a negative error code. */
int miugks_timing(miugks_ctx* ctx, int cap, const char** names, int* launches, double* ms, double* bytes);

/* Sizes: cells, fluid cells, velocities, levels. */
int miugks_sizes(const miugks_ctx* ctx, int* nc, int* n_fluid, int* nk, int* n_levels);

#ifdef __cplusplus
}
#endif

#endif /* MIUGKS_H */
