/*
 * tdks.h -- C ABI of the MI355X (gfx950) real-time TDKS propagator with
 * two-step Brillouin-zone sampling.
 *
 * Method: Sato, "Two-step Brillouin zone sampling for efficient computation
 * of electron dynamics in solids", arXiv:2112.00920.
 *   - TDKS equation for the periodic parts u_bk of the Bloch orbitals,
 *     i d/dt u_bk = h_k(t) u_bk                                  (Sec. II.A, Eq. 1)
 *   - h_k(t) = [p + k + A(t)]^2/2 + v_ion + v_Hxc[rho]          (Eq. 2)
 *   - rho = sum_b BZ-average |u_bk|^2                            (Eq. 3)
 *   - J = -(1/Omega) sum_b BZ-average <u_bk| pi_k |u_bk>,
 *     pi_k = (1/i)[r, h_k]                                       (Eqs. 5-6)
 *   - BZ average on a (shifted) Monkhorst-Pack grid             (Eqs. 7-8, 10)
 *   - two-step scheme: N_H independent sub-simulations on shifted coarse
 *     grids, observables averaged over them                      (Sec. II.B, Eq. 9)
 *
 * Numerics (the paper defers them to its production code; fixed here):
 *   - real-space grid N1 x N2 x N3 along the lattice rows a_1, a_2, a_3;
 *     4th-order finite differences (+-2 neighbours, periodic) for the kinetic
 *     operator in the periodic-part gauge:
 *       T_kappa = -1/2 L - i kappa . grad_FD + |kappa|^2 / 2, kappa = k + A(t);
 *   - v_ion = Gaussian local potential + s and p Kleinman-Bylander projectors
 *     per atom (Gaussian radial shape rc, shifted cut at Rc);
 *   - v_Hxc = Hartree (Poisson by discrete Fourier transform, G = 0 and Nyquist
 *     planes zeroed) + Slater exchange + Perdew-Zunger 81 correlation;
 *   - propagator: explicit Taylor expansion of exp(-i h dt) to 4th order with
 *     h evaluated at A(t_n + dt/2) and v_Hxc[rho(t_n)];
 *   - the current after step n uses A(t_{n+1}).
 *
 * Conventions
 *   - Atomic units throughout (bohr, hartree, a.u. of time).
 *   - Orbital arrays passed across this ABI are complex128 (interleaved
 *     re, im doubles) laid out [k][band][i3][i2][i1] (i1 fastest), normalised
 *     to sum_r |u|^2 dV = 1 with dV = Omega / (N1 N2 N3).
 *   - Fractional k are in units of the reciprocal vectors b_d
 *     (a_d . b_e = 2 pi delta_de) and must already be wrapped the way the
 *     caller wants them (the FD Hamiltonian is not periodic in k).
 *   - Every function returns TDKS_OK (0) or a negative error code; the
 *     message of the last error on the calling thread is tdks_last_error().
 *   - A context is not thread-safe.  All device work of a context is ordered
 *     on one internal HIP stream, which waits for the caller's stream at entry
 *     and which the caller's stream waits for at exit of every call.
 *   - Pointers marked HOST are host memory; pointers marked "where" are host
 *     (TDKS_HOST) or device (TDKS_DEVICE) memory of the context's GPU.  Input
 *     arrays are borrowed for the duration of the call only (copied).
 */
#ifndef TDKS_H
#define TDKS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define TDKS_OK 0
#define TDKS_E_ARG (-1)         /* invalid argument or descriptor            */
#define TDKS_E_OOM (-2)         /* device allocation failed                   */
#define TDKS_E_HIP (-3)         /* HIP runtime error                          */
#define TDKS_E_STATE (-4)       /* call not valid in the context's state      */
#define TDKS_E_NUMERIC (-5)     /* numeric health check failed (tdks_check)    */
#define TDKS_E_UNSUPPORTED (-6) /* size or option outside the built kernels   */

/* precision of the propagation arithmetic */
#define TDKS_FP64 0       /* complex128 orbitals and arithmetic                   */
#define TDKS_FP32_MIXED 1 /* complex64 orbitals, FP32 stencil/potential/projector
                             arithmetic; FP64 density, current, Hxc and norms   */

/* Hartree-exchange-correlation coupling */
#define TDKS_HXC_SCF 0    /* v_Hxc recomputed from rho after every step          */
#define TDKS_HXC_FROZEN 1 /* v_Hxc fixed to the array given in the descriptor    */
#define TDKS_HXC_NONE 2   /* v_Hxc = 0                                           */

/* propagators (tdks_options.propagator) */
#define TDKS_PROP_TAYLOR 0 /* explicit Taylor-4 step, h with v_Hxc[rho(t_n)]      */
#define TDKS_PROP_PC 1     /* predictor-corrector: v_Hxc at the mid-step (SCF)    */

/* memory location flags */
#define TDKS_HOST 0
#define TDKS_DEVICE 1

/* current read-out modes */
#define TDKS_PER_INSTANCE 0
#define TDKS_PER_GROUP 1

/* One pseudopotential species (Sec. II.A: local part + non-local projectors). */
typedef struct tdks_species {
    double D;  /* depth of the local Gaussian D exp(-r^2 / (2 w^2)) (Ha)        */
    double w;  /* width of the local Gaussian (bohr); images within 15 w count  */
    double rc; /* Gaussian radius of the KB projectors (bohr)                   */
    double Rc; /* shifted-cut radius of the KB projectors (bohr); must be below
                  half of the shortest lattice translation                      */
    double Es; /* KB energy of the s channel (Ha)                               */
    double Ep; /* KB energy of the three p channels (Ha)                        */
} tdks_species;

/* One independent TDDFT simulation (one sub-simulation of the two-step scheme,
 * Sec. II.B procedure step 3, or one plain-method run). */
typedef struct tdks_instance_desc {
    double lattice[3][3];        /* rows a_1, a_2, a_3 (bohr)                      */
    int grid[3];                 /* N1, N2, N3                                     */
    int n_atoms;
    const double *atom_frac;     /* HOST [n_atoms][3] fractional positions         */
    const int *atom_species;     /* HOST [n_atoms] index into species               */
    int n_species;
    const tdks_species *species; /* HOST [n_species]                                */
    int n_k;
    const double *k_frac;        /* HOST [n_k][3] fractional k (units of b_d)       */
    const double *k_weight;      /* HOST [n_k] BZ weights, or NULL for 1/n_k (Eq. 7) */
    int n_bands;
    const double *occ;           /* HOST [n_bands] occupations, or NULL for 2.0     */
    int group;                   /* two-step group id (averaged in PER_GROUP mode)  */
    const double *v_hxc_frozen;  /* HOST [N3][N2][N1], required iff TDKS_HXC_FROZEN */
} tdks_instance_desc;

/* Tiling of the instances of one shape (an autotuner's result per shape class): applies to
 * the instances whose grid equals `grid` and whose lattice and band count match; the first
 * matching rule wins, and fields left 0 fall back to tdks_options.  All instances of one grid
 * shape and lattice kind share one block size and occupancy target. */
typedef struct tdks_tiling_rule {
    int grid[3];          /* N1, N2, N3                                             */
    int nonorth;          /* 1 non-orthogonal lattices, 0 orthogonal, -1 either     */
    int n_bands;          /* band count it applies to, 0 any                         */
    int block_size;       /* threads per workgroup (0 = automatic)                   */
    int waves_per_simd;   /* 2 or 4 (0 = automatic)                                  */
    int bands_per_group;  /* bands per workgroup (0 = all)                           */
    int k_per_group;      /* k-points per workgroup (0 = automatic)                  */
} tdks_tiling_rule;

typedef void *(*tdks_alloc_fn)(size_t bytes, void *user);
typedef void (*tdks_free_fn)(void *ptr, void *user);

typedef struct tdks_options {
    int precision;        /* TDKS_FP64 or TDKS_FP32_MIXED                         */
    double dt;            /* time step (a.u.)                                      */
    int taylor_order;     /* must be 4                                             */
    int hxc_mode;         /* TDKS_HXC_SCF / _FROZEN / _NONE                        */
    void *stream;         /* caller's hipStream_t, or NULL for the null stream     */
    tdks_alloc_fn alloc;  /* device allocator, or NULL for hipMalloc               */
    tdks_free_fn free;    /* matching free, or NULL for hipFree                    */
    void *alloc_user;     /* passed to alloc/free                                  */
    int bands_per_group;  /* bands propagated by one workgroup (0 = all, or, for a
                             grid shape with fewer work items than the GPU's 256
                             compute units, the bands split in halves down to 8)  */
    int k_per_group;      /* k-points per workgroup (0 = 4 for instances with at
                             least 256 k-points when the context has at least
                             16384 (k, band group) items, else 1)                 */
    int block_size;       /* threads per workgroup (0 = automatic: the z-segments'
                             threads rounded up to whole waves, a block of more
                             than 8 waves padded to 16; a request at least the
                             segments' count, up to 1024, is taken as given)      */
    int graph_steps;      /* steps captured per HIP graph (0 = 16; <0 disables)    */
    int waves_per_simd;   /* occupancy target of the propagation kernel: 2 or 4
                             (0 = automatic); selects the register budget          */
    int propagator;       /* TDKS_PROP_TAYLOR (default) or TDKS_PROP_PC            */
    int norm_stride;      /* per-orbital norm check every norm_stride steps (0 = off;
                             the charge is checked every step regardless)          */
    int record_stride;    /* record the current every record_stride-th step (0 = 1) */
    const tdks_tiling_rule *tiling_rules; /* HOST [n_tiling_rules], read by tdks_create only;
                                             per-shape overrides of the fields above    */
    int n_tiling_rules;
} tdks_options;

typedef struct tdks_ctx tdks_ctx;

/* Fills *opt with defaults (FP64, dt = 0.02, order 4, SCF, automatic tiling). */
void tdks_default_options(tdks_options *opt);

/* Creates a context holding n_inst independent instances (Sec. II.B step 3:
 * one TDDFT simulation per shift; instances may differ in cell, grid, k-count
 * and band count).  Builds the grid, the local potential, the projector
 * support tables and the k tables on the host, allocates the device memory
 * through opt->alloc, and returns the context in *out.
 * Errors: E_ARG (bad descriptor, e.g. Rc too large for the cell), E_OOM,
 * E_HIP, E_UNSUPPORTED (an axis outside 4..32 points or more than 8192 grid
 * points, more than 64 atoms, more than 4095 projector column images or 65535
 * support entries, a grid whose orbital does not fit the 160 KB of LDS of one
 * workgroup beside its small tables, taylor_order != 4).  FP64 grids whose
 * per-column-image tables do not fit beside the orbital (20^3, 16x16x32) keep those
 * tables in device memory, one slice per work item (a slower path).  All of these are detected on the host
 * before any device call.  E_ARG also for tiling rules that give one shape class two
 * different block sizes or occupancy targets. */
int tdks_create(const tdks_instance_desc *inst, int n_inst, const tdks_options *opt,
                tdks_ctx **out);

/* Releases all device memory and the internal stream.  NULL is allowed. */
void tdks_destroy(tdks_ctx *ctx);

/* Thread-local message of the last error ("" if none). */
const char *tdks_last_error(void);

/* Loads the orbitals of instance `inst` (complex128, [k][band][i3][i2][i1],
 * `where` = TDKS_HOST or TDKS_DEVICE), rounding to complex64 for
 * TDKS_FP32_MIXED.  Then computes rho (Eq. 3), v_Hxc (SCF mode), and the
 * current before the field, J_pre = J(A = 0) (Sec. III.A: delta J is measured
 * against J(t < 0)).  Resets the step counter of the context.
 * Errors: E_ARG, E_HIP. */
int tdks_load_orbitals(tdks_ctx *ctx, int inst, const void *u, int where);

/* Numeric health check (checked on the device inside every step, no host work).  The
 * Taylor-4 step multiplies the squared norm of each eigencomponent of the Hermitian h_kappa by
 * |T4(-i x)|^2 = 1 - x^6/72 + x^8/576, x = dt lambda (Eq. 1 expanded to 4th order): <= 1 for
 * |x| <= 2 sqrt 2, decreasing in |x| below sqrt 6.  Every step checks, per instance, that the
 * current J^{n+1} (Eq. 5) and the charge Q = sum_k w_k sum_b f_b ||u_bk||^2 (the integral of
 * Eq. 3) are finite and that Q0 F_1 ... F_n (1 - tol) <= Q <= Q0 (1 + tol), Q0 = Q at the load,
 * F_m = that factor at x = |dt| lambda_max(A(t_m + dt/2)) with lambda_max a bound of |lambda|
 * (kinetic bound at kappa = k + A, |v_loc|, the KB operator norms, and 5 Ha for |v_Hxc|);
 * tol = 1e-9 (FP64) or 1e-4 (FP32_MIXED).  With norm_stride > 0 every norm_stride-th step also
 * checks each orbital's norm against the same bounds times its norm at the load.  The first
 * violation of each instance is recorded on the device. */

/* Advances every instance by n_steps Taylor-4 steps (Eq. 1) under the uniform
 * vector potential table A_tab (HOST, [n_steps][2][3]: A(t_n + dt/2) used in
 * h for step n, and A(t_{n+1}) used for the current recorded after it).
 * With TDKS_PROP_PC and SCF Hxc each step is a predictor-corrector pair: a
 * predictor Taylor-4 step from u^n with v_Hxc[rho(t_n)] whose density gives
 * v~ (its orbitals are not stored), then the step from u^n with
 * (v_Hxc[rho(t_n)] + v~) / 2; twice the propagation work, and the Hxc coupling
 * becomes second order in dt.  With frozen or no Hxc the two propagators are
 * the same step.  The
 * current J^{n+1} (Eq. 5) of every instance is recorded after every
 * record_stride-th step.  Enqueued asynchronously (HIP graphs of opt->graph_steps
 * steps); the host does no per-step work.  The health record is copied to the host
 * asynchronously at the end of the call.  Errors: E_STATE (an instance not loaded),
 * E_ARG, E_OOM (trace growth), E_HIP, E_NUMERIC (the health record of an earlier
 * call had arrived by the start of this one and shows a violation: nothing is
 * enqueued; the message names the instance, the step and the check). */
int tdks_step(tdks_ctx *ctx, int n_steps, const double *A_tab);

/* Allocation-free variant of tdks_step for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * Advances every instance by n_steps steps exactly as tdks_step does, with the same
 * kernels, but the A table comes from the caller's device memory (A_dev, DEVICE
 * [n_steps][2][3], as A_tab), the currents go to the caller's device buffer (j_dev,
 * DEVICE [n_inst][n_steps][3]: J^{n+1} of each step of the call, the current itself, not
 * delta J; subtract tdks_current_pre; record_stride does not apply), and the per-work-item
 * partial sums of the density and current live in one static device array of 32 MiB per
 * GPU (held until the process ends) instead of the context's buffers.  The call allocates
 * nothing (no hipMalloc, hipFree, pinned or host staging) and does not synchronise: it only
 * enqueues kernels on the context's stream, fenced against the caller's stream as every call
 * is, so a caller may capture it into a HIP graph.  Every step overwrites the partial sums
 * it reads, so the array needs no clearing; all calls on one GPU share it, so calls that
 * overlap on one GPU (contexts driven from different streams or threads) race and must be
 * serialised by the caller.  The health check runs with the step-independent floor 0.25 of
 * |T4(-i x)|^2 for its lower bound (the A table is not read on the host).  After such a
 * call tdks_current returns E_STATE until the next load (these steps have no trace rows).
 * Errors: E_ARG (null buffers, n_steps < 0, another device current), E_STATE (an instance
 * not loaded), E_UNSUPPORTED (the context's partial sums, sum over instances of
 * (8 N_g + 32) bytes per work item with 256-byte alignment, exceed 32 MiB; tdks_step has no
 * such limit), E_HIP. */
int tdks_step_noalloc(tdks_ctx *ctx, int n_steps, const double *A_dev, double *j_dev);

/* Waits for the context's work and returns E_NUMERIC if any instance failed the health
 * check since its load (the message names the first such instance, the step counted from
 * the load, the check, and for an orbital check its k and band), else TDKS_OK.  info
 * (HOST [n_inst], may be NULL) receives each instance's record: 0 = healthy, else
 * step << 32 | (k n_bands + band + 1) << 4 | code (orbital field 0 for the charge checks;
 * code 1 non-finite current or charge, 2 / 3 charge above / below its bounds, 4 / 5 an
 * orbital norm above / below them).  A load or tdks_ground_state clears the records of
 * the instances it sets.  Errors: E_ARG, E_HIP, E_NUMERIC. */
int tdks_check(tdks_ctx *ctx, unsigned long long *info);

/* Number of steps taken since the last load (a load resets it); the current is
 * recorded for steps_done / record_stride of them. */
int tdks_steps_done(tdks_ctx *ctx);

/* Ground-state preparation (the runs of Sec. III start from the Kohn-Sham
 * ground state; delta J is measured against it).  Starting from the loaded
 * (or present) orbitals of every instance, runs n_iter iterations of:
 *   1. the propagator of Eq. (1) at imaginary time, exp(-tau h_k) with A = 0,
 *      by the same Taylor-4 expansion and kernels as tdks_step
 *      (w_m = (-tau/m) h w_{m-1}), filtering the bands towards the lowest
 *      eigenvectors of h_k;
 *   2. Cholesky orthonormalisation of the bands of each k (S = U^H U dV =
 *      L L^H, U <- U L^{-H}, FP64);
 *   3. the density rho_out (Eq. 3) and the residual sum |rho_out - rho_in| dV;
 *   4. SCF mode: linear mixing rho_in <- (1 - mix) rho_in + mix rho_out and
 *      v_Hxc[rho_in]; FROZEN / NONE modes keep their potential (rho_in <-
 *      rho_out).
 * rho_in starts as the density of the starting orbitals.  With every band
 * occupied, rho, J and the total energy depend only on the span of the bands,
 * which converges to the lowest n_bands eigenvectors when h_k has a gap above
 * them.  Afterwards rho, v_Hxc and J_pre are those of the final orbitals (as
 * after tdks_load_orbitals) and the step counter is reset.  residual (HOST
 * [n_inst], may be NULL) receives the last iteration's residual per instance.
 * n_iter = 0 only recomputes rho, v_Hxc and J_pre (residual receives zeros).
 * The first call allocates its buffers through the context's allocator: one
 * FP64 density partial per k-point of every instance (8 N_g n_k bytes each),
 * the mixing's input density and the residuals.  Synchronises.
 * Stability: the Taylor-4 filter is bounded for tau lambda_max(h_k) < 2.78; the
 * call rejects tau whose kinetic bound alone exceeds 2.5 / tau.
 * Errors: E_ARG (n_iter < 0, tau <= 0 or too large, mix outside (0, 1]),
 * E_STATE (an instance not loaded), E_UNSUPPORTED (more than 32 bands),
 * E_NUMERIC (linearly dependent bands: S not positive definite; orbitals of
 * that k are left unchanged), E_OOM, E_HIP. */
int tdks_ground_state(tdks_ctx *ctx, int n_iter, double tau, double mix, double *residual);

/* Copies the induced current delta J^n = J^n - J_pre for n = s, 2s, ..., R s
 * (s = record_stride, R = steps_done / s) into out (HOST).  mode TDKS_PER_INSTANCE:
 * [n_inst][R][3]; TDKS_PER_GROUP: [n_groups][R][3], the plain mean over the
 * instances of each group in ascending group id (Eq. 9 / procedure step 4).  cap
 * is the capacity of out in doubles; *n_written receives the number written.
 * Synchronises.  Errors: E_ARG (cap too small), E_NUMERIC (the health check of
 * tdks_check failed, or a non-finite value; the message names the instance),
 * E_HIP. */
int tdks_current(tdks_ctx *ctx, int mode, double *out, size_t cap, size_t *n_written);

/* J_pre of every instance, HOST out[n_inst][3].  Synchronises. */
int tdks_current_pre(tdks_ctx *ctx, double *out);

/* Current of the present orbitals of every instance at kappa = k + A
 * (A HOST [3]), without propagating: out HOST [n_inst][3].  Synchronises. */
int tdks_current_at(tdks_ctx *ctx, const double *A, double *out);

/* Density rho (FP64, HOST out [N3][N2][N1]) of instance inst after the last
 * step (or load).  Synchronises. */
int tdks_density(tdks_ctx *ctx, int inst, double *rho_out);

/* Diagnostics (not on the timed path). */

/* v_Hxc in use for the next step of instance inst, HOST out [N3][N2][N1]. */
int tdks_vhxc(tdks_ctx *ctx, int inst, double *out);

/* Local potential v_loc of instance inst, HOST out [N3][N2][N1]. */
int tdks_vloc(tdks_ctx *ctx, int inst, double *out);

/* Present orbitals of instance inst as complex128 [k][band][i3][i2][i1]. */
int tdks_get_orbitals(tdks_ctx *ctx, int inst, void *u_out, int where);

/* Norms sum_r |u|^2 dV (FP64) of instance inst, HOST out [k][band]. */
int tdks_norms(tdks_ctx *ctx, int inst, double *out);

/* One application hw = h_kappa w (Eq. 2) for every k and band of instance
 * inst, with kappa = k + A (A HOST [3]) and the present v_Hxc; w and hw are
 * complex128 [k][band][i3][i2][i1] in `where` memory.  Uses the propagation
 * kernel's stencil, potential and projector code path. */
int tdks_apply_h(tdks_ctx *ctx, int inst, const void *w, void *hw, const double *A, int where);

/* Advances every instance by n_steps exactly like tdks_step, but launches the
 * step's kernels one by one (no graph) with HIP events recorded on the
 * context's stream around them, and returns the mean device time per step in
 * out (HOST [3], milliseconds): [0] the propagation kernels (Taylor-4 step with
 * density and current partials; predictor and corrector for TDKS_PROP_PC),
 * [1] the reduction, Hxc, mid-step potential and counter kernels, [2] the
 * whole step.  Synchronises.  Same errors as tdks_step. */
int tdks_time_kernels(tdks_ctx *ctx, int n_steps, const double *A_tab, double *out);

/* Tiling actually used by the first grid shape (the first instance's): threads per
 * workgroup, length of the z-column segment each thread owns, occupancy target (waves
 * per SIMD), bands and k-points per workgroup (of the first work item), and the number
 * of workgroups per step (all shapes).  Outputs may be NULL. */
int tdks_tiling(tdks_ctx *ctx, int *block, int *zl, int *waves_per_simd, int *bands_per_group,
                int *k_per_group, int *n_groups);

#ifdef __cplusplus
}
#endif

#endif /* TDKS_H */
