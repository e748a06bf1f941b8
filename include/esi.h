/*
 * esi.h -- C ABI of the MI355X (gfx950) hot path of time-domain extended
 * source waveform inversion (ESI), after Yang & Zhou, "Algorithmic analysis
 * towards time-domain extended source waveform inversion" (arXiv 2211.06300).
 *
 * The library solves, shot by shot, the ESI normal equation
 *     (S^T S + beta B^T B) q = S^T d                       (eq. normalewi, Sec. 2.3)
 * with S = R A^{-1} the modelling operator of the constant-density acoustic
 * equation A(m) u = (1/v^2) d_t^2 u - Laplacian u (eq. wave, Sec. 2.1), and it
 * forms the adjoint-state gradient <lambda, (dA/dm) u> (eq. gradewi, Sec. 2.3).
 *
 * Conventions shared by every call
 * --------------------------------
 *  * Grid: a physical grid nz x nx (2D) or nz x ny x nx (3D), spacing dx, with
 *    an absorbing layer of nb cells added OUTSIDE it on every side (Sec. 4.1
 *    asks for an absorbing boundary that also removes the free surface).  The
 *    layer is a damping term eta(x) u_t, eta = eta_max sum_d (delta_d/nb)^2.
 *    Beyond the padded grid the field is zero.
 *  * Scheme: O(dt^2, dx^8) (Sec. 4.1).  With c = v^2 dt^2, k = eta dt / 2,
 *        (1+k) u^{n+1} = 2 u^n - (1-k) u^{n-1} + c (L u^n + P q^n),
 *        d^n = R u^{n+1},      n = 0 .. nt-1,   u^{-1} = u^0 = 0,
 *    so q^n enters at step n and d^n is the sample at time (n+1) dt.  The
 *    adjoint runs the same recurrence backward in time with R^T d^j injected.
 *  * Positions are 0-based physical cell indices, (ix, iz) in 2D and
 *    (ix, iz, iy) in 3D.
 *  * Dense wavefield-sized vectors (extended sources q, CG vectors, adjoint
 *    outputs) are float32 [nshots][nt][nz][(ny)][nx], x fastest, physical
 *    grid only.  Data are float32; the traces of one shot are [nt][nrec_s]
 *    and shots follow each other in the order of geom.rec_ptr (CSR): within
 *    a call on shots [shot0, shot0+nshots) the data of shot s start at
 *    element nt * (rec_ptr[s] - rec_ptr[shot0]).
 *  * Model: m = 1/v^2.  Gradients are with respect to m on the physical grid
 *    (multiply by -2/v^3 for the gradient with respect to v).
 *  * Annihilator: B(x) = |x - x_s| / dx + b_eps (distance in cells), the
 *    choice of Sec. 4 with a small positive number added at the source.
 *  * Inner products are plain sums over cells and steps.
 *
 * Memory and streams: every pointer named "device" is device memory on the
 * plan's device, owned by the caller, float32 and contiguous unless stated.
 * The plan owns only what it derives (coefficients, wavefield rings, data
 * and reduction scratch, per-tile injection lists); it grows that scratch on
 * demand with hipMalloc and frees it in esi_plan_destroy (esi_forward_noalloc
 * is the one call that never allocates).  All work is
 * queued on the stream given at plan creation; calls return once the work is
 * queued, except esi_cg_solve, which waits for each iteration's residual norms
 * to decide convergence.
 *
 * Errors: every call returns an esi_status_t; nothing aborts and no C++
 * exception crosses the boundary.  Arguments are validated before any work is
 * queued.  esi_last_error() returns a text for the last failure on the
 * calling thread.  A plan must not be used from two threads at once.
 */
#ifndef ESI_H
#define ESI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct esi_plan_s* esi_plan_t;
typedef struct esi_unet_s* esi_unet_t;

typedef enum {
    ESI_OK = 0,
    ESI_ERR_ARG = 1,        /* null pointer, bad enum, bad shot range */
    ESI_ERR_SHAPE = 2,      /* inconsistent sizes or positions outside the grid */
    ESI_ERR_CFL = 3,        /* v_max dt / dx beyond the stability limit */
    ESI_ERR_OOM = 4,        /* device allocation failed */
    ESI_ERR_HIP = 5,        /* a HIP runtime call or kernel launch failed */
    ESI_ERR_BREAKDOWN = 6,  /* CG: p^T N p <= 0 */
    ESI_ERR_NONFINITE = 7   /* CG: non-finite scalar */
} esi_status_t;

enum { ESI_SRC_POINT = 0, ESI_SRC_DENSE = 1 };
enum { ESI_GRAD_PENALTY = 0, ESI_GRAD_ADJOINT = 1, ESI_GRAD_SEED = 2, ESI_GRAD_SEED_REUSE = 3 };

typedef struct {
    int32_t ndim;       /* 2 or 3 */
    int32_t nz, nx, ny; /* physical grid; ny must be 1 when ndim == 2 */
    int32_t nb;         /* absorbing-layer width in cells, >= 4 */
    int32_t nt;         /* number of time steps, >= 1 */
    double dx, dt;      /* metres, seconds */
    double eta_max;     /* peak damping (1/s); < 0: 3 v_max ln(1000) / (2 nb dx); 0: off */
    double beta;        /* penalty weight of eq. (esi), >= 0 */
    double b_eps;       /* annihilator offset in cells, > 0 when beta > 0 */
} esi_grid_t;

typedef struct {
    int32_t nshots;
    const int32_t* src;     /* host [nshots][ndim] source cells */
    const int64_t* rec_ptr; /* host [nshots+1], rec_ptr[0] = 0, non-decreasing */
    const int32_t* rec;     /* host [rec_ptr[nshots]][ndim] receiver cells */
    const int32_t* window;  /* host [nshots][2] or NULL (2D only): shot s propagates on the
                               physical columns [window[2s], window[2s+1]) alone (its aperture),
                               with the absorbing layer around that window (the model beyond the
                               window edge fills the layer, edge copies beyond the grid); its
                               source and receivers must lie in the window.  Dense vectors keep
                               the whole-grid layout and are zero outside the window.  Launches
                               cover only the tiles that meet a window, so a batch of shots of
                               uneven aperture costs the sum of their windows.  NULL: every
                               shot uses the whole grid. */
} esi_geom_t;

/*
 * Create a plan for one grid, acquisition and velocity model.
 *   vel:    device [nz][(ny)][nx] velocity in m/s (copied; the caller keeps it).
 *   stream: hipStream_t to queue work on (NULL = default stream).
 * Checks the CFL limit of the 8th-order scheme (v_max dt/dx <= 0.5547 in 2D,
 * 0.4529 in 3D) -> ESI_ERR_CFL.  Geometry arrays are copied.
 */
esi_status_t esi_plan_create(esi_plan_t* plan, const esi_grid_t* grid, const esi_geom_t* geom,
                             const float* vel, void* stream);

/* Replace the velocity model (device [nz][(ny)][nx]); same checks as creation.
 * eta_max keeps the value fixed at plan creation. */
esi_status_t esi_plan_set_model(esi_plan_t plan, const float* vel);

/* Release the plan and every buffer it owns (waits for its stream). */
esi_status_t esi_plan_destroy(esi_plan_t plan);

/* Text of the last error on this thread ("" if none).  Valid until the next call. */
const char* esi_last_error(void);

/*
 * Forward modelling d = S q (Sec. 2.1 eq. fwi / eq. wave; S = R A^{-1}, Sec. 2.2).
 *   src_kind ESI_SRC_POINT: src = device [nshots][nt] wavelets, injected at each
 *            shot's source cell (the physical source f).
 *   src_kind ESI_SRC_DENSE: src = device [nshots][nt][phys] extended source q
 *            (eq. newq2), injected on every physical cell.
 *   data:    device output, [nshots] x [nt][nrec_s] (CSR layout above).
 */
esi_status_t esi_forward(esi_plan_t plan, int32_t shot0, int32_t nshots, int32_t src_kind,
                         const float* src, float* data);

/*
 * Adjoint modelling S^T d = A^{-T} R^T d (eq. FWI_lambda; the CG right-hand side
 * "by adjoint modelling", Sec. 3).
 *   data: device input, CSR layout; receivers sharing a cell add up.
 *   out:  device output [nshots][nt][phys].
 */
esi_status_t esi_adjoint(esi_plan_t plan, int32_t shot0, int32_t nshots, const float* data,
                         float* out);

/*
 * Matrix-free normal operator N p = S^T S p + beta B^T B p (eq. axb, Sec. 3:
 * forward modelling with p as the source, receiver extraction, adjoint
 * modelling, plus the pointwise beta B^2 p).
 *   p, Ap: device [nshots][nt][phys] (must not overlap).
 *   pAp:   device double [nshots] output p . Np per shot, or NULL.
 */
esi_status_t esi_normal_apply(esi_plan_t plan, int32_t shot0, int32_t nshots, const float* p,
                              float* Ap, double* pAp);

typedef struct {
    int32_t iters;       /* out: largest number of iterations done by a shot */
    int32_t* shot_iters; /* host [nshots] out, or NULL */
    double* res_hist;    /* host [nshots][max_iter+1] out, or NULL: ||r_k|| / ||r_0|| of
                            the recursively updated residual; unused entries set to -1 */
    /* esi_fpcg_solve only (ignored by esi_cg_solve; set to NULL there): */
    int32_t* shot_fallback; /* host [nshots] out, or NULL: iteration after which the first
                               preconditioner was given up, -1 if never */
    int32_t* shot_cg;       /* host [nshots] out, or NULL: iteration after which plain CG
                               took over, -1 if never */
    const float* stat_xref; /* device [nshots][nt][phys] reference solution, or NULL */
    float* stat_out;        /* device [max_iter+1][nshots][2][phys], or NULL: for the iterate
                               x_k and residual r_k of every iteration k reached, the cell maps
                               a = sum_t r_k^2 and c = sum_t r_k (x_ref - x_k) (training pairs
                               of the learned preconditioner); entries of iterations a shot did
                               not reach are left untouched */
} esi_cg_report_t;

/*
 * Conjugate gradients (Algorithm 1, Sec. 3) on eq. (normalewi), one independent
 * system per shot, x_0 = 0.  Each shot stops after the iteration in which
 * ||r_{k+1}|| < rtol ||r_0||, or after max_iter iterations.  Vectors are
 * float32; dot products and step lengths are float64.
 *   d_obs: device data (CSR layout).
 *   x:     device [nshots][nt][phys] output (the extended source).
 *   work:  device float32 scratch of 3 * nshots * nt * phys elements (r, p, Np).
 *   rep:   host report, may be NULL.
 * Returns ESI_ERR_BREAKDOWN if p.Np <= 0 or ESI_ERR_NONFINITE on a non-finite
 * scalar; x then holds the last finished iterate.
 */
esi_status_t esi_cg_solve(esi_plan_t plan, int32_t shot0, int32_t nshots, const float* d_obs,
                          float* x, float* work, int32_t max_iter, double rtol,
                          esi_cg_report_t* rep);

/*
 * State of a CG solve between iterations, for saving a solve and resuming it
 * later (Algorithm 1's (x, r, p, r.r, k) with the per-shot bookkeeping).  The
 * vectors stay in the caller's buffers: x = x_k, work[0] = r_k, work[1] =
 * p_{k-1} (work as in esi_cg_solve).  Host arrays, [nshots] unless stated:
 */
typedef struct {
    int32_t k;          /* iterations done */
    double* rr0;        /* ||r_0||^2 */
    double* rr;         /* ||r_k||^2 */
    double* beta;       /* beta_{k-1}: the next direction is r_k + beta p_{k-1} */
    int32_t* iterating; /* 1 if the shot stopped only at the iteration limit */
    int32_t* iters;     /* iterations done by the shot */
    int32_t* status;    /* ESI_OK, ESI_ERR_BREAKDOWN or ESI_ERR_NONFINITE of the shot */
    double* res_hist;   /* [nshots][hist_cap]: ||r_j|| / ||r_0||, j <= k (later entries -1) */
    int32_t hist_cap;   /* row length of res_hist */
} esi_cg_state_t;

/*
 * esi_cg_solve with save and resume.  resume = NULL starts from x_0 = 0 as
 * esi_cg_solve does; otherwise the solve continues from the state (d_obs is
 * not read; x and work hold the saved vectors; 1 <= resume->k <= max_iter;
 * hist_cap >= k + 1) up to max_iter iterations in all, the shots flagged
 * `iterating` taking part.  save, if not NULL (hist_cap >= max_iter + 1),
 * receives the state after the last iteration, with p_{k-1} copied into
 * work[1].  A solve paused after K iterations and resumed to K' gives the
 * same x, r and residual history bit for bit as one solve of K' iterations
 * (graph replay, esi_plan_set_cg_graph, is not used while resuming).
 * Errors as esi_cg_solve; ESI_ERR_ARG for an inconsistent state.
 */
esi_status_t esi_cg_solve_state(esi_plan_t plan, int32_t shot0, int32_t nshots, const float* d_obs,
                                float* x, float* work, int32_t max_iter, double rtol,
                                const esi_cg_state_t* resume, esi_cg_state_t* save, esi_cg_report_t* rep);

/*
 * Adjoint-state gradient with respect to m = 1/v^2, summed over the shots and
 * ADDED to grad_m (device [phys]):
 *   g(x) = sum_n lambda^n(x) v(x)^2 (L u^n + P q^n)(x),   u = A^{-1} q,
 * where v^2 (L u^n + q^n) is the discrete (dA/dm) u (eq. gradewi, Sec. 2.3).
 *   ESI_GRAD_PENALTY: lambda = beta B^T B q (Algorithm 2); src = q (dense).
 *                     One forward pass; no wavefield storage.  data unused.
 *   ESI_GRAD_ADJOINT: lambda = S^T (d_obs - S q) (eq. ewiadj); src = q (dense),
 *                     data = d_obs.
 *   ESI_GRAD_SEED:    gradients of a loss L(d), d = S q, given data = dL/dd:
 *                     adds -sum_n (S^T G)^n (dA/dm) u^n to grad_m and, when
 *                     grad_src is not NULL, writes dL/dq to grad_src
 *                     ([nshots][nt] for a point source, [nshots][nt][phys] for a
 *                     dense one).  src_kind as in esi_forward.
 *   ESI_GRAD_SEED_REUSE: as SEED, but the forward pass is not run again: the
 *                     wavefield checkpoints saved by the last esi_forward_ckpt
 *                     call are used (same shot0, nshots, src_kind, src pointer
 *                     and ckpt_every, model unchanged since); ESI_ERR_ARG if the
 *                     plan holds no such checkpoints.
 *   ckpt_every: 0 stores (dA/dm)u for every step (nshots*nt*phys floats of plan
 *               scratch); K > 0 stores two time levels every K steps and
 *               recomputes each K-step segment during the backward pass.
 */
esi_status_t esi_gradient(esi_plan_t plan, int32_t shot0, int32_t nshots, int32_t mode,
                          int32_t src_kind, const float* src, const float* data,
                          float* grad_m, float* grad_src, int32_t ckpt_every);

/*
 * Forward modelling as esi_forward that also keeps wavefield checkpoints (two
 * time levels every ckpt_every steps, 2 * ceil(nt/K) padded fields per shot of
 * plan scratch) for a following esi_gradient(ESI_GRAD_SEED_REUSE) call: the
 * differentiation pattern in which the forward pass stores checkpoints and the
 * backward pass recomputes K-step segments (the storage remedy of Sec. 5.1).
 * Any esi_gradient call in ADJOINT, SEED or SEED_REUSE mode, or another
 * esi_forward_ckpt call, releases the checkpoints.  ckpt_every >= 1.
 */
esi_status_t esi_forward_ckpt(esi_plan_t plan, int32_t shot0, int32_t nshots, int32_t src_kind,
                              const float* src, float* data, int32_t ckpt_every);

/*
 * Forward modelling as esi_forward that allocates no device memory, for
 * callers that cannot call hipMalloc: work under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  Same arguments, results
 * (bit for bit) and errors as esi_forward.
 *   The wavefield ring of the call (4 padded fields per shot) lives in a
 *   fixed device array of the library, 64 MiB per GPU, held until the
 *   process ends; nshots * 4 * (padded storage field) * 4 bytes beyond that
 *   -> ESI_ERR_SHAPE (call with fewer shots).  The array is cleared by each
 *   call before use.
 *   Every call on one GPU uses that GPU's one array: calls that overlap in
 *   time on the same GPU (two streams, two threads, two plans) race and give
 *   wrong results; serialise them.
 *   The plan must come from esi_plan_create (which builds the tile lists this
 *   call needs and looks up the array's address on the device).
 */
esi_status_t esi_forward_noalloc(esi_plan_t plan, int32_t shot0, int32_t nshots, int32_t src_kind,
                                 const float* src, float* data);

/*
 * Penalty weight of the plan (Sec. 2.2-2.3, Table compare):
 *   ESI_WEIGHT_ANNIHILATOR (default): B = |x - x_s| / dx + b_eps, the ESI
 *     annihilator (eq. esi);
 *   ESI_WEIGHT_IDENTITY: B = I, the WRI penalty (eq. wridSf); the normal
 *     operator becomes S^T S + beta I (eq. normalwri).
 * It applies to every later call (normal operator, CG, PENALTY gradients).
 * esi_fpcg_solve refuses identity-weight plans (its cell scales model the
 * annihilator).  ESI_ERR_ARG for another kind.
 */
enum { ESI_WEIGHT_ANNIHILATOR = 0, ESI_WEIGHT_IDENTITY = 1 };
esi_status_t esi_plan_set_weight(esi_plan_t plan, int32_t kind);

/*
 * Data residual of the physical source, the WRI right-hand side data
 * (eq. wridSf / eq. normalwri):  d_res = d_obs - S f, with f = the point
 * wavelets ([nshots][nt], device) at the shots' sources.  d_obs and d_res are
 * device data arrays of the shots (layout as esi_forward's data; d_res may
 * alias d_obs).  esi_cg_solve(d_res) then solves (S^T S + beta W) q =
 * S^T (d - S f).
 */
esi_status_t esi_data_residual(esi_plan_t plan, int32_t shot0, int32_t nshots,
                               const float* wavelet, const float* d_obs, float* d_res);

/*
 * WRI gradient with respect to m = 1/v^2 (Sec. 2.2, Table compare), summed
 * over the shots and ADDED to grad_m (device [phys]):
 *   g(x) = sum_n lambda^n(x) v(x)^2 (L u^n + P(f + q)^n)(x),  u = A^{-1}(f + q),
 * with f the point wavelets ([nshots][nt], device) and q the dense extension
 * ([nshots][nt][phys], device).
 *   ESI_GRAD_PENALTY: lambda = beta W q (W = B^T B of the plan; I for WRI):
 *                     one forward pass, no storage, d_obs unused.  Equal to
 *                     ADJOINT when q solves the normal equation.
 *   ESI_GRAD_ADJOINT: lambda = S^T (d_obs - S(f + q)): the gradient of
 *                     J_WRI at fixed q.  ckpt_every as in esi_gradient.
 * ESI_ERR_ARG for other modes or null pointers.
 */
esi_status_t esi_wri_gradient(esi_plan_t plan, int32_t shot0, int32_t nshots, int32_t mode,
                              const float* wavelet, const float* q, const float* d_obs,
                              float* grad_m, int32_t ckpt_every);

/*
 * Penalty parameter beta of the plan (Sec. 2.4): used by every later call.
 * ESI_ERR_ARG unless finite.  The normal operator is positive definite only
 * for beta > 0 (Sec. 2.3); a negative beta makes it indefinite, and CG then
 * stops with ESI_ERR_BREAKDOWN at the first p.Np <= 0, x holding the last
 * iterate it finished.
 */
esi_status_t esi_plan_set_beta(esi_plan_t plan, double beta);

/*
 * The outer loop of Algorithm 2 (nested loops for variable projection between
 * m = 1/v^2 and q), run by the library:
 *   per outer iteration: the inner loop (CG on the normal equation, Algorithm 1,
 *   cg_iters iterations or cg_rtol) for every shot; the PENALTY gradient
 *   (lambda = beta W q, u = A^{-1} q); a direction -H g with H the L-BFGS
 *   inverse-Hessian approximation (two-loop recursion, lbfgs_mem pairs, a pair
 *   kept when s'y > 0); a backtracking line search (step halved at most ls_max
 *   times) with the Armijo condition J(m_t) <= J(m) + c1 g'(m_t - m) on the
 *   model clipped to [v_min, v_max].  Without curvature pairs the first trial
 *   is -g scaled to max |dm| = first_step * max m.
 *   J(m) = sum over shots of 1/2 ||S q - d||^2 + beta/2 ||B q||^2 for the inner
 *   loop's q (eq. esi).  With wavelet != NULL (WRI, Sec. 2.2; set the plan's
 *   weight to ESI_WEIGHT_IDENTITY) the inner loop solves for q with
 *   right-hand side S^T(d - S f), u = A^{-1}(f + q) and
 *   J = 1/2 ||S(f + q) - d||^2 + beta/2 ||q||^2 (eq. wridSf).
 *   beta_rule ESI_BETA_DISCREPANCY (Sec. 2.4, Sec. 4.3): before each outer
 *   iteration, while the relative data misfit ||S q - d|| / ||d|| is below
 *   misfit_lo beta is multiplied by beta_factor, while above misfit_hi it is
 *   divided by it (at most beta_tries changes; each re-solves and clears the
 *   L-BFGS memory).  ESI_BETA_FIXED keeps the plan's beta.
 * d_obs: device data of the shots (layout of esi_forward); wavelet: device
 * [nshots][nt] or NULL; vel: device [phys], the starting model on entry and
 * the last accepted model on return (the plan is left at that model and at
 * the final beta); grad_mask: device [phys] multiplying the gradient, or NULL;
 * x: device [shot_group][nt][phys] and work: device [3][shot_group][nt][phys],
 * the inner solves' vectors (shots are solved shot_group at a time).  The
 * library allocates its FP64 model-space vectors (2 lbfgs_mem + 6 of [phys])
 * per call.
 * The inner solver is Algorithm 1 (ESI_INNER_CG) or, for ESI, the flexible CG
 * of esi_fpcg_solve preconditioned by the analytic cell scale
 * 1 / (beta B^2 + inner_gamma), recomputed whenever beta changes
 * (ESI_INNER_FCG_SCALE): the inner loop then converges in far fewer
 * iterations, as Sec. 3 asks of it; or the data-space CG of esi_ds_cg_solve
 * (ESI_INNER_DATASPACE, cg_iters iterations of the data-space system).
 * rep (optional) receives the counts and, through its non-NULL host arrays,
 * the histories.  Returns ESI_ERR_ARG for bad options; a failed line search is
 * not an error (rep->status = 1, vel = the last accepted model).
 */
enum { ESI_BETA_FIXED = 0, ESI_BETA_DISCREPANCY = 1 };
enum { ESI_INNER_CG = 0, ESI_INNER_FCG_SCALE = 1, ESI_INNER_DATASPACE = 2 };
typedef struct {
    int32_t outer_iters;   /* N_outer >= 0 */
    int32_t cg_iters;      /* inner CG iterations >= 1 */
    double cg_rtol;        /* inner stopping tolerance (0: run cg_iters) */
    int32_t shot_group;    /* shots per inner solve, 1..nshots */
    int32_t lbfgs_mem;     /* >= 1 */
    int32_t ls_max;        /* line-search trials >= 1 */
    double armijo_c1;      /* in (0, 1) */
    double first_step;     /* > 0 */
    double v_min, v_max;   /* 0 < v_min < v_max (m/s); v_max must meet the CFL limit */
    int32_t beta_rule;     /* ESI_BETA_FIXED or ESI_BETA_DISCREPANCY */
    double misfit_lo, misfit_hi;   /* discrepancy band, 0 <= lo <= hi */
    double beta_factor;    /* > 1 */
    int32_t beta_tries;    /* >= 0 */
    int32_t inner;         /* ESI_INNER_CG: Algorithm 1; ESI_INNER_FCG_SCALE: esi_fpcg_solve with
                              the cell scale 1 / (beta B^2 + inner_gamma) (ESI only);
                              ESI_INNER_DATASPACE: esi_ds_cg_solve (2D, beta > 0) */
    double inner_gamma;    /* > 0 */
} esi_invert_opts_t;
typedef struct {
    int32_t outer_done;    /* accepted outer iterations */
    int32_t evals;         /* objective evaluations */
    int32_t status;        /* 0: ran outer_iters iterations, 1: a line search failed */
    double beta_final;
    double* J;             /* host [outer_iters + 1] or NULL: J at the accepted models */
    double* misfit;        /* host [outer_iters + 1] or NULL: relative data misfit there */
    double* beta;          /* host [outer_iters + 1] or NULL: beta of each J */
    double* beta_iter;     /* host [outer_iters] or NULL: beta of each outer iteration */
    double* step;          /* host [outer_iters] or NULL: accepted step lengths */
    int32_t* trials;       /* host [outer_iters] or NULL: line-search trials */
} esi_invert_report_t;
esi_status_t esi_invert(esi_plan_t plan, int32_t shot0, int32_t nshots, const float* d_obs,
                        const float* wavelet, float* vel, const float* grad_mask, float* x,
                        float* work, const esi_invert_opts_t* opts, esi_invert_report_t* rep);

/*
 * Frequency-domain ESI with time-domain modelling (Sec. 5.2, eq. (dtft),
 * eq. (idtft), eq. (normaldtft)), 2D and 3D plans.  Frequency vectors are device
 * float32 arrays [nshots][nf][phys][2] of (re, im) pairs: the DTFT
 * (F u)_m = sum_n u_n exp(+j 2 pi f_m n dt) of a [nt][phys] field at the
 * plan's nf frequencies.  G s = (1/nt) Re sum_m s_m exp(-j 2 pi f_m n dt) is
 * the inverse (the real part: the modelling needs a real source), so that
 * G = F^* / nt under the real inner product Re sum conj(a) b.  The time loops
 * never store a whole time axis: G feeds the forward pass as its source and F
 * of the adjoint field accumulates in complex float32 slices (per step inside
 * the stencil kernel, or per block of steps: esi_plan_set_dtft_block).
 *
 * esi_dtft_set_freqs: nf (1..32) frequencies in Hz (host array); the plan
 *   keeps the twiddle table and F G (a 2nf x 2nf real matrix).  ESI_ERR_ARG
 *   for a bad count or a negative or non-finite frequency.
 * esi_dtft_normal_apply: Mp = F (S^T S + beta W) G p with the plan's weight W;
 *   pMp (device double [nshots], nullable) = Re p^H M p.  p and Mp must not
 *   alias.
 * esi_dtft_rhs: b = F S^T G F d_obs (the data represented through the inverse
 *   DTFT of their DTFT); d_obs as in esi_forward.
 * esi_dtft_cg_solve: Algorithm 1 on M x = F S^T G F d_obs with the real inner
 *   product, per shot, FP64 dots and step lengths; x: frequency vectors; work:
 *   three more; rep and errors as esi_cg_solve.
 * esi_dtft_to_time: q = G x, device [nshots][nt][phys].
 * esi_dtft_gradient: Algorithm 2's PENALTY gradient with the time-domain source
 *   q = G x formed on the fly (lambda = beta W q, u = A^{-1} q), summed over
 *   the shots and ADDED to grad_m (device [phys]).
 * Each returns ESI_ERR_ARG when esi_dtft_set_freqs has not been called, or on
 * a 3D plan set to meet the slices at every step (esi_plan_set_dtft_block
 * with 0: that path lives inside the 2D stencil kernel).
 */
esi_status_t esi_dtft_set_freqs(esi_plan_t plan, int32_t nf, const double* freqs_hz);
esi_status_t esi_dtft_normal_apply(esi_plan_t plan, int32_t shot0, int32_t nshots, const float* p,
                                   float* Mp, double* pMp);
esi_status_t esi_dtft_rhs(esi_plan_t plan, int32_t shot0, int32_t nshots, const float* d_obs, float* b);
esi_status_t esi_dtft_cg_solve(esi_plan_t plan, int32_t shot0, int32_t nshots, const float* d_obs,
                               float* x, float* work, int32_t max_iter, double rtol,
                               esi_cg_report_t* rep);
esi_status_t esi_dtft_to_time(esi_plan_t plan, int32_t shot0, int32_t nshots, const float* x, float* q);
esi_status_t esi_dtft_gradient(esi_plan_t plan, int32_t shot0, int32_t nshots, const float* x,
                               float* grad_m);

/*
 * How the DTFT calls above meet the frequency slices in their time loops.
 * block = 0: inside the step kernel at every step (G x forms each step's
 * source from the slices; F of the adjoint field is accumulated into them).
 * block = K > 0 (default 64): per K steps, one kernel forms the K steps'
 * sources into a K-step buffer that the forward pass reads as its dense
 * source, and one kernel folds the K adjoint fields that the adjoint pass
 * wrote into that buffer into the slices, so each slice crosses HBM once per
 * K steps instead of at every step.  Each cell's operations run in the same
 * order either way: the results are identical bit for bit.  The plan keeps a
 * buffer of nshots x min(K, nt) x nz x nx floats.  ESI_ERR_ARG for a null
 * plan or block outside 0..1024.
 */
esi_status_t esi_plan_set_dtft_block(esi_plan_t plan, int32_t block);

/*
 * Data-space solution of the normal equation (Sec. 5.1, eq. (vd), eq. (wv),
 * eq. (q): the Sherman-Morrison-Woodbury route), beta > 0:
 *   CG (Algorithm 1, per shot, FP64 dots) on (beta I + S W^{-1} S^T) w = v,
 *   v = S W^{-1} S^T d, with W = B^T B of the plan (I for ESI_WEIGHT_IDENTITY);
 *   then, when q != NULL, q = (beta W)^{-1} S^T (d - w).
 * An application of S W^{-1} S^T is an adjoint pass that stores the adjoint
 * field (plan scratch, nshots * nt * phys floats) and a forward pass with that
 * field times W^{-1} as its source.  For WRI pass d - S f (esi_data_residual).
 * d, w: device data of the shots (layout of esi_forward's data); w receives
 * the synthetic data.  q: device [nshots][nt][phys] or NULL.  work: device,
 * 3 data vectors.  rep as esi_cg_solve (residuals of the data-space system).
 * 2D and 3D plans.  ESI_ERR_ARG for beta <= 0, shots without receivers, or
 * null pointers; ESI_ERR_BREAKDOWN / ESI_ERR_NONFINITE as esi_cg_solve.
 */
esi_status_t esi_ds_cg_solve(esi_plan_t plan, int32_t shot0, int32_t nshots, const float* d, float* w,
                             float* q, float* work, int32_t max_iter, double rtol, esi_cg_report_t* rep);

/*
 * Storage of the adjoint field inside esi_ds_cg_solve (Sec. 5.1 names
 * checkpointing as the remedy for the memory that field takes).  every = 0
 * (default): the field of the whole time axis stays resident (nshots * nt *
 * phys floats).  every = K > 0: one adjoint pass saves the adjoint state every
 * K steps (nshots * ceil(nt / K) * 2 padded fields), and before the forward
 * pass runs each K-step segment the segment's field is recomputed from the
 * checkpoint above it into a K-step buffer (nshots * K * phys floats): one
 * more adjoint propagation per operator application, results identical bit
 * for bit.  ESI_ERR_ARG for a null plan or every < 0.
 */
esi_status_t esi_plan_set_ds_ckpt(esi_plan_t plan, int32_t every);

/*
 * Chain rule from m = 1/v^2 to v: grad_v = -2 grad_m / v^3 on the physical
 * grid (device [phys] each; grad_v may alias grad_m).
 */
esi_status_t esi_grad_velocity(esi_plan_t plan, const float* vel, const float* grad_m,
                               float* grad_v);

/*
 * Time blocking of the 2D kernels: 2 (default) advances two time steps per
 * launch wherever a call allows it (the wavefield state then crosses HBM once
 * per two steps; launch shape ESI_LAUNCH_TWO_STEP_32), 1 advances one step per
 * launch (ESI_LAUNCH_ONE_STEP).  Results are identical bit for bit either way.
 * Returns ESI_ERR_ARG for other values.
 */
esi_status_t esi_plan_set_time_block(esi_plan_t plan, int32_t steps);

/*
 * Launch shapes of the time loops, the autotuner's candidates:
 *   ESI_LAUNCH_ONE_STEP (1): one time step per launch (2D: 64 x 32 tiles;
 *   3D: 64 x 16 columns, 32-plane chunks);
 *   ESI_LAUNCH_TWO_STEP_32 (2, default), _24 (3), _40 (4): two time steps per
 *   launch on 56-column tiles of 32, 24 or 40 rows (2D), or on 56 x 24 columns
 *   and 64-plane chunks (3D, shape 2 only); the wavefield state crosses HBM
 *   once per two steps and the first step runs on the tile grown by one
 *   stencil radius.
 * Every shape gives the same wavefield, data, dense outputs and gradients bit
 * for bit; float64 dot products sum their per-tile partials over a different
 * tiling, so CG results agree to rounding.  Time-loop variants the shapes of
 * 24 and 40 rows do not cover run on 32-row tiles.
 */
enum { ESI_LAUNCH_ONE_STEP = 1, ESI_LAUNCH_TWO_STEP_32 = 2, ESI_LAUNCH_TWO_STEP_24 = 3,
       ESI_LAUNCH_TWO_STEP_40 = 4 };

/* Set the launch shapes of forward-type and adjoint-type loops (1 .. 4; 3D:
 * 1 or 2).  ESI_ERR_ARG otherwise. */
esi_status_t esi_plan_set_launch_shape(esi_plan_t plan, int32_t forward, int32_t adjoint);

/*
 * Autotuner of the launch shape.  For the plan's grid and a batch of nshots
 * shots it times every candidate shape (2D: the four above; 3D: 1 and 2), after a
 * warm-up run of each, with the plan's hipEvent profiling, and keeps the
 * fastest for forward-type and for adjoint-type loops separately.
 *   p, Ap device [nshots][nt][phys] (contents irrelevant; Ap is overwritten):
 *     the candidates are timed on one application of the normal operator;
 *   p = Ap = NULL: on a point-source forward pass over the first min(nt, 64)
 *     steps and a gradient's adjoint pass over the last ones, injecting
 *     receiver data and correlating with a two-slot (dA/dm)u store (for
 *     batches whose wavefield-sized vectors are too large to allocate, e.g.
 *     the gradients of many shots of long records; the store and the per-shot
 *     images are plan scratch, 3 x nshots x physical cells floats).
 * Choices and timings are cached per process for (ndim, padded shape,
 * nshots, nt, the shots' apertures, timing kind); force != 0 measures again.
 * choice: host int[2] out (forward, adjoint launch shape) or NULL.
 */
esi_status_t esi_plan_autotune(esi_plan_t plan, int32_t shot0, int32_t nshots, const float* p,
                               float* Ap, int32_t force, int32_t* choice);

/* The candidate table of the plan's last esi_plan_autotune call (also when it
 * came from the cache): count rows (host out); for i < min(cap, count) the
 * shape and the milliseconds of its forward-type and adjoint-type loops (host
 * arrays [cap] out). */
esi_status_t esi_plan_tune_table(esi_plan_t plan, int32_t cap, int32_t* count, int32_t* shape,
                                 double* fwd_ms, double* adj_ms);

/*
 * CG iterations (Algorithm 1) replayed from captured HIP graphs.  With
 * enable != 0, esi_cg_solve runs iteration 0 directly and captures iterations
 * 1 and 2 once (one graph per parity of the iteration index, since the
 * direction and N p buffers alternate); later iterations and later solves with
 * the same shots, buffers, iteration limit and tolerance replay them.  The
 * stopping test, the residual history and the retirement of converged shots
 * run on the device, so the host only polls one counter per iteration.
 * Results are identical bit for bit to enable = 0.  The plan owns a stream
 * for capture and replay, ordered after its own stream by events.
 */
esi_status_t esi_plan_set_cg_graph(esi_plan_t plan, int32_t enable);

/*
 * CG iterations (Algorithm 1) with the residual update fused into the normal
 * operator; on by default.  In every iteration p_k . N p_k is
 * taken as ||S p_k||^2 + beta ||B p_k||^2 from the forward pass (the two are
 * equal in exact arithmetic, S being the receiver data of the forward
 * modelling and N = S^T S + beta B^2), so alpha_k is known before the adjoint
 * pass, which updates r in place instead of storing N p_k for a separate
 * pass.  enable = 0 restores the separate pass (p_k . N p_k then comes from
 * N p_k itself); the two agree to float32 rounding, not bit for bit.  The
 * flexible and preconditioned solvers keep the separate pass.
 * Errors: ESI_ERR_ARG for a null plan.
 */
esi_status_t esi_plan_set_cg_rfuse(esi_plan_t plan, int32_t enable);

/*
 * Kernel timing (the tracing facility of the library).  With profiling on,
 * every time loop of a call is bracketed by a pair of hipEvents on the plan's
 * stream; esi_plan_profile_read waits for them and reports, per time-step
 * kernel variant, the number of launches and the elapsed milliseconds of the
 * loops that ran it (kernel time plus the gaps between its launches).  The
 * variant is a bit set of fused work (source kind, recording, injection,
 * outputs, CG fusion, correlation) whose meaning is given by the ESI_K_*
 * values below; ESI_K_TWO_STEP marks launches that advance two steps, and
 * bits 16-18 of such a variant hold its launch shape (ESI_LAUNCH_*; 2D tile
 * height, or the 3D two-step kernel).  Turning profiling on (enable != 0)
 * clears the counters.
 */
enum {
    ESI_K_SRC_POINT = 1, ESI_K_SRC_DENSE = 2, ESI_K_CG_FUSE = 4, ESI_K_INJ = 8,
    ESI_K_GATHER = 16, ESI_K_OUT = 32, ESI_K_NORMAL = 64, ESI_K_PENALTY = 128,
    ESI_K_STORE = 256, ESI_K_CORR = 512, ESI_K_SRC_REC = 1024, ESI_K_TWO_STEP = 32768
};
esi_status_t esi_plan_profile(esi_plan_t plan, int32_t enable);
/* Fills up to `cap` entries; *count receives the number of variants seen.
 * flags: host uint32 [cap]; launches: host int64 [cap]; ms: host double [cap];
 * shot_launches: host int64 [cap], launches weighted by the shots each covered. */
esi_status_t esi_plan_profile_read(esi_plan_t plan, int32_t cap, int32_t* count, uint32_t* flags,
                                   int64_t* launches, int64_t* shot_launches, double* ms);

/*
 * Flexible conjugate gradients with truncation 1 (FCG(1), Notay 2000) on
 * eq. (normalewi), one system per shot, x_0 = 0 (2D plans).  The paper solves
 * the normal equation with plain CG (Algorithm 1) and leaves preconditioning
 * open (Sec. 4.2, Sec. 6); this call adds it.  Per iteration: z_k = M(r_k),
 * alpha = p.r / p.Np, x += alpha p, r -= alpha Np, beta = -z.Np / p.Np,
 * p = z + beta p.  The preconditioner scales the residual cell by cell,
 * z = s r, with s = s0 exp(o):
 *   scale: s0, device [nshots][phys], or NULL for s0 = 1;
 *   net:   o = Net(features) from the residual's per-cell energy (see
 *          esi_precond_features), or NULL for o = 0; the network must take
 *          Hp x Wp images (nz, nx rounded up to multiples of 8) in batches of
 *          at least nshots.  It runs on r_0 and then every net_every-th
 *          iteration (net_every = 0: once, so the preconditioner is fixed
 *          and the iteration is preconditioned CG).
 * Both NULL is CG with beta in Hestenes-Stiefel form.
 * A shot gives up its preconditioner when z.r <= 0 or is not finite, or when
 * ||r|| has not reached a new best by 1 % for 20 iterations: with a network
 * it drops the correction (s = s0), then, and without one at once, it falls
 * back to plain CG (s = 1); each switch restarts the direction at p = z and
 * the 20-iteration window.  Stopping as esi_cg_solve: ||r_{k+1}|| < rtol ||r_0|| of the
 * recursively updated residual, or max_iter.
 *   d_obs, x, work, max_iter, rtol: as esi_cg_solve (work: 3 vectors).
 *   rep: as esi_cg_solve, plus shot_fallback and the training maps
 *        (stat_xref / stat_out) when given.
 * Errors as esi_cg_solve; ESI_ERR_ARG for 3D plans, ESI_ERR_SHAPE for a
 * network of the wrong size.
 */
esi_status_t esi_fpcg_solve(esi_plan_t plan, int32_t shot0, int32_t nshots, const float* d_obs,
                            float* x, float* work, int32_t max_iter, double rtol, esi_unet_t net,
                            int32_t net_every, const float* scale, esi_cg_report_t* rep);

/*
 * The analytic cell scale of the flexible solver, s0(x) = 1 / (beta B(x)^2 +
 * gamma) per shot, B = |x - x_s| / dx + b_eps in cells: the inverse of the
 * penalty weight of eq. (esi) (the term beta B^T B of eq. normalewi) with
 * gamma standing in for the part S^T S adds.  It is the base scale of
 * esi_fpcg_solve and esi_precond_features.
 *   out: device [nshots][phys] float32 out (computed in float64, rounded once).
 * 2D annihilator-weight plans only (ESI_ERR_ARG otherwise); gamma > 0.
 */
esi_status_t esi_precond_scale(esi_plan_t plan, int32_t shot0, int32_t nshots, double gamma, float* out);

/*
 * Network input of the preconditioner for `nshots` shots of a 2D plan, on
 * images padded to Hp x Wp (multiples of 8, at least nz x nx; zero outside
 * the grid): channel 0 = log(1 + rms_t(r) / mean_x rms_t(r)) with
 * rms_t(r) = sqrt(a/nt), channel 1 = v / 3000 m/s, channel 2 = log(B) / 4
 * (B = |x - x_s| / dx + eps, in cells).
 *   a:    device [nshots][phys], a = sum_t r^2 of each shot's residual.
 *   cmap: device [nshots][phys] or NULL (c = sum_t r e of a training pair).
 *   base: device [nshots][phys] base scale s0, or NULL for 1.
 *   xin:  device [nshots][3][Hp][Wp] out; apad, cpad: device [nshots][Hp][Wp]
 *         out or NULL: a s0^2 and cmap s0 zero-padded (the training maps of
 *         the correction exp(o) on top of s0, see esi_unet_loss_grad).
 */
esi_status_t esi_precond_features(esi_plan_t plan, int32_t shot0, int32_t nshots, const float* a,
                                  const float* cmap, const float* base, int32_t Hp, int32_t Wp,
                                  float* xin, float* apad, float* cpad);

/* ------------------------------------------------------------------------
 * Learned preconditioner network.  The paper leaves preconditioning of its CG
 * open (Sec. 4.2; Sec. 6 calls for a preconditioner that cuts the number of
 * inner iterations); this library's is a four-level U-Net whose output o(x)
 * scales the residual cell by cell, z = exp(o) r, recomputed every iteration
 * of a flexible CG (esi_fpcg_solve).
 *
 * Architecture (channels 16/32/64/128, 3x3 convolutions with zero padding,
 * ReLU, 2x2 average pooling, 2x2 stride-2 transposed convolutions, skip
 * concatenation [upsampled, skip], 1x1 output):
 *   c1a 3->16, c1b 16->16 | pool | c2a 16->32, c2b 32->32 | pool |
 *   c3a 32->64, c3b 64->64 | pool | c4a 64->128, c4b 128->128 |
 *   u3 128->64, d3a 128->64, d3b 64->64 | u2 64->32, d2a 64->32, d2b 32->32 |
 *   u1 32->16, d1a 32->16, d1b 16->16 | out 16->1.
 * Flat float32 parameter vector, layers in that order, each layer's weights
 * then its bias; weight layouts conv3x3 [co][ci][3][3], convT [ci][co][2][2],
 * out [1][16].  482033 parameters.
 * Arithmetic: weights and activations bfloat16 (round to nearest even), bias,
 * accumulation, the output o and all parameter gradients float32; gradients
 * of activations are bfloat16.  Adam keeps float32 master parameters.
 * The network runs on the stream given at creation; calls are asynchronous
 * unless they return a host value.  A network handle is not thread-safe.
 * ------------------------------------------------------------------------ */

/* Number of parameters of the network (482033). */
int64_t esi_unet_num_params(void);

/* Network for images of H x W pixels (multiples of 8) and batches of up to
 * max_batch images; activation memory about 700 B per pixel per image.
 * Parameters start at zero: set them with esi_unet_set_params.
 * ESI_ERR_SHAPE for other sizes, ESI_ERR_OOM when allocation fails. */
esi_status_t esi_unet_create(esi_unet_t* net, int32_t H, int32_t W, int32_t max_batch, void* hip_stream);
esi_status_t esi_unet_destroy(esi_unet_t net);

/* Copy the float32 parameters in (theta: host or device [P]) and clear the
 * Adam moments; get copies them out.  Both synchronise the network's stream. */
esi_status_t esi_unet_set_params(esi_unet_t net, const float* theta);
esi_status_t esi_unet_get_params(esi_unet_t net, float* theta);

/* o = Net(x) for `batch` images: x device [batch][3][H][W] float32 (NCHW),
 * o device [batch][H][W] float32. */
esi_status_t esi_unet_forward(esi_unet_t net, const float* x, float* o, int32_t batch);

/* Loss of the scaling preconditioner and its gradient.  For each image s,
 * with a = sum_t r^2 and c = sum_t r e (device [batch][H][W], zero on padding
 * pixels), L_s = w_s sum_x (a e^{2o} - 2 c e^{o}): the squared error of
 * exp(o) r against e up to a constant; L = mean_s L_s.  weight: device
 * [batch] w_s, or NULL for the default of each image (esi_unet_loss_weights),
 * which scales the loss so that 0 is no correction and -1 the best single
 * scale.  Writes dL/dtheta into grad (device [P], overwritten) and L into
 * *loss (host, may be NULL; non-NULL synchronises). */
esi_status_t esi_unet_loss_grad(esi_unet_t net, const float* x, const float* a, const float* c,
                                const float* weight, int32_t batch, float* grad, double* loss);

/* Default loss weights of `batch` images of npix pixels on `hip_stream`:
 * w = sum a / (sum c)^2, 0 when sum c <= 0 (a, c device [batch][npix], w
 * device [batch] out).  Tiles cut from a larger image take the whole image's
 * weight. */
esi_status_t esi_unet_loss_weights(const float* a, const float* c, int32_t batch, int64_t npix,
                                   float* w, void* hip_stream);

/* One Adam step (Kingma & Ba) on the master parameters with gradient grad
 * (device [P]); step counts from 1.  clip_norm > 0 first scales the gradient
 * to norm at most clip_norm (computed on the device). */
esi_status_t esi_unet_adam(esi_unet_t net, const float* grad, float lr, float beta1, float beta2,
                           float eps, int32_t step, float clip_norm);

#ifdef __cplusplus
}
#endif

#endif /* ESI_H */
