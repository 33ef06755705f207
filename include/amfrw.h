/*
 * amfrw.h -- C ABI of libamfrw: AMFR-W time stepping on every component grid of the (modified)
 * sparse-grid combination technique for the SABR-LIBOR market model PDE, on AMD Instinct MI355X
 * (gfx950).  Method: Lopez-Salas, Perez-Rodriguez, Vazquez, "AMFR-W numerical methods for solving
 * high dimensional SABR/LIBOR PDE models", arXiv 2408.00559.
 *
 * Conventions shared by every call
 *   - Every call returns amf_status; nothing throws or aborts across the ABI.  On failure
 *     amf_last_error() returns a message (thread-local, valid until the next call on the thread).
 *   - Streams are passed as `void*` and are hipStream_t handles (0 = the null stream).  Enqueueing
 *     calls are asynchronous: results are valid once the stream has been synchronised.
 *   - Device memory is caller-owned.  A plan keeps host metadata only; its device state lives in
 *     one workspace of amf_plan_info.workspace_bytes bytes bound with amf_plan_bind, which must stay
 *     allocated until all enqueued work that uses it has completed.
 *   - A plan is not used from two host threads at once.  Plans never share device memory.
 *   - Grid vectors on the device hold INNER nodes only (every index j_i in 1..M_i, Section 3 of the
 *     paper), in the plan precision, axis 1 fastest: the element of unit u at multi-index j sits at
 *     unit_offset(u) + sum_i (j_i - 1) * prod_{k<i} M_k.  Lower-face (Outer) values are implied:
 *     the payoff for solution vectors, 0 for stage increments.  Axis d-1 is the volatility V.
 *     With AMF_BC_DIRICHLET the nodes j_i = M_i of a rate axis are stored as well but are boundary
 *     data: the solution holds the payoff there and stage increments hold 0.
 */
#ifndef AMFRW_H
#define AMFRW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AMF_ABI_VERSION 2
#define AMF_MAX_D 8        /* descriptor capacity; kernels are built for d = 2..6 */
#define AMF_MAX_STAGES 6

typedef enum {
    AMF_OK = 0,
    AMF_E_INVALID = 1,     /* a descriptor or argument is out of range          */
    AMF_E_UNSUPPORTED = 2, /* valid request this build does not implement        */
    AMF_E_NOMEM = 3,       /* host allocation failed                             */
    AMF_E_HIP = 4,         /* a HIP runtime call or kernel launch failed         */
    AMF_E_NUMERIC = 5,     /* non-finite result (results are still written)      */
    AMF_E_STATE = 6        /* call order violated (e.g. solve before bind)       */
} amf_status;

typedef enum { AMF_FP64 = 0, AMF_FP32 = 1 } amf_precision;

typedef enum {
    AMF_PAYOFF_CAPLET = 0,   /* tau_1 (F_1 - K)^+ (Section 2)                                    */
    AMF_PAYOFF_SWAPTION = 1  /* max{ sum_i tau_i (F_i - K) / prod_{l<=i} (1 + tau_l F_l), 0 }   */
} amf_payoff;

/* Conditions on the upper faces F_i = F_i^max of the rate axes (Section 2).  The lower faces carry
 * the payoff and V = V^max is homogeneous Neumann in both. */
typedef enum {
    AMF_BC_NEUMANN = 0,      /* homogeneous Neumann, eq (bound1): the paper's choice               */
    AMF_BC_DIRICHLET = 1     /* the payoff, eq (bound1_0): the upper rate faces are boundary data,  */
                             /* so a rate axis of M_i intervals has M_i - 1 unknowns               */
} amf_boundary;

/* Matrix W of the W-method (row-s). */
typedef enum {
    AMF_W_AMF = 0,           /* the AMF-refined W of eq (Wmat1): per stage the chain of directional */
                             /* solves, the refinement and a second chain (eq amfrw)               */
    AMF_W_LOWER = 1          /* W = P, the lower triangle (diagonal included) of the semi-discrete  */
                             /* matrix in the theta_0 order: a fixed number of Gauss-Seidel sweeps  */
                             /* of the theta-method written as a W-method (Section 4.2, eq (GS))    */
} amf_w_matrix;

/* One pricing instance: the data of the PDE (mmNd) in time-to-maturity form, with coefficients
 * (coef_diff), (coef_mix), (coef_adv), the domain of Section 3 and the boundary conditions: the
 * payoff on the lower faces, homogeneous Neumann at V = V^max, and on the upper faces of the rate
 * axes the kind `boundary` selects.  Copied at amf_plan_create; the caller may free it afterwards. */
typedef struct {
    uint32_t struct_size;                       /* = sizeof(amf_problem)                          */
    int32_t d;                                  /* N: d-1 forward rates plus V, 2 <= d <= 6      */
    int32_t payoff;                             /* amf_payoff                                     */
    int32_t boundary;                           /* amf_boundary                                   */
    double beta;                                /* elasticity, 0 <= beta <= 1                     */
    double sigma;                               /* volatility of V (>= 0)                         */
    double alpha[AMF_MAX_D - 1];                /* alpha_i >= 0                                   */
    double phi[AMF_MAX_D - 1];                  /* F_i - V correlation, |phi_i| <= 1             */
    double tau[AMF_MAX_D - 1];                  /* accrual periods tau_i >= 0                     */
    double rho[(AMF_MAX_D - 1) * (AMF_MAX_D - 1)]; /* rho[i*(AMF_MAX_D-1)+j], unit diagonal      */
    double x_max[AMF_MAX_D];                    /* F_1^max .. F_{d-1}^max, V^max (> 0)           */
    double maturity;                            /* T > 0, the PDE horizon                         */
    double strike;                              /* K                                              */
    double x_eval[AMF_MAX_D];                   /* evaluation point, inside the domain            */
    double discount;                            /* price = discount * u(T, x_eval)                */
} amf_problem;

/* s-stage W-method, eq (row-s): (I - theta dt W) K_r = dt F(Y_n + sum_j a_rj K_j) + sum_j q_rj K_j,
 * Y_{n+1} = Y_n + sum_r b_r K_r, with W chosen by w_matrix (stages as eq (amfrw) for the AMF W).
 * a and q are stored row-major [r*AMF_MAX_STAGES + j] for j < r; 1 <= stages <= AMF_MAX_STAGES. */
typedef struct {
    uint32_t struct_size;
    int32_t stages;
    double a[AMF_MAX_STAGES * AMF_MAX_STAGES];
    double q[AMF_MAX_STAGES * AMF_MAX_STAGES];
    double b[AMF_MAX_STAGES];
    double theta;
    double nu;                                  /* AMF parameter of (Wmat1) (AMF_W_AMF only)      */
    int32_t w_matrix;                           /* amf_w_matrix                                   */
    int32_t reserved;                           /* 0                                              */
} amf_scheme;

/* Either one full grid (M_i = 2^levels[i]) or the combination technique at level n with offset psi:
 * eq (standardCombTechnique) for psi = 0, eq (modifiedCombTechnique) for psi > 0. */
typedef struct {
    uint32_t struct_size;
    int32_t full_grid;                          /* 1: levels[] is used; 0: n and psi are used     */
    int32_t levels[AMF_MAX_D];                  /* 0 <= level <= 20                               */
    int32_t n;                                  /* d - 1 <= n, n + psi <= 20, n + d psi <= 30     */
    int32_t psi;                                /* 0 <= psi <= 8                                  */
} amf_grid_spec;

typedef struct amf_plan amf_plan;

typedef struct {
    int64_t n_problems;
    int64_t n_units;                  /* (problem, component grid) pairs                           */
    int64_t inner_points;             /* sum over units of prod M_i                                */
    int64_t stage_updates_per_solve;  /* inner_points * stages * steps (x3 with Richardson)        */
    uint64_t workspace_bytes;
    uint64_t state_offset;            /* byte offset of the stored Y - g inside the workspace      */
    uint64_t vector_bytes;            /* bytes of one grid vector: all units, each unit's offset   */
                                      /* rounded up to a multiple of 64 elements and of             */
                                      /* min(M_1, 1024) (padding is never read)                     */
    int32_t d;
    int32_t precision;                /* amf_precision                                             */
    int32_t n_steps;
    int32_t richardson;
} amf_plan_info;

/* ABI version of the library (AMF_ABI_VERSION). */
int32_t amf_abi_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char* amf_last_error(void);

/* The paper's AMFR-W2 (coef_W2): a21 = 2/3, q21 = -4/3, b = (5/4, 3/4), theta = (3 + sqrt 3)/6,
 * third order; nu = theta (the paper leaves nu unprinted; nu = theta reproduces its tables). */
amf_status amf_scheme_amfrw2(amf_scheme* out);

/* The theta-method (thetamet) with `stages` Gauss-Seidel sweeps (GS) as a W-method (Section 4.2):
 * W = P, a_rj = theta, q_rj = -1, b_r = 1; second order at theta = 1/2 for stages >= 2.
 * AMF_E_INVALID unless 0 < theta <= 1 and 1 <= stages <= AMF_MAX_STAGES. */
amf_status amf_scheme_theta_gs(double theta, int32_t stages, amf_scheme* out);

/* Build a plan: enumerate the component grids of `grid` for each of the n_probs problems (all with
 * the same d), lay out the device workspace, tabulate the 1-D coefficient factors of (coef_diff),
 * (coef_mix), (coef_adv) in FP64 and round them once to the plan precision.  dt = maturity/n_steps
 * per problem.  richardson = 1 also runs 2*n_steps and combines prices as (8 P_fine - P_coarse)/7
 * (fourth order in time from a third-order scheme such as AMFR-W2).  Errors: AMF_E_INVALID for
 * out-of-range descriptors (d, levels, n < d-1, psi, beta, correlations, boundary, x_eval outside
 * the domain, steps < 1, stages, w_matrix, theta, nu), AMF_E_UNSUPPORTED for the W = P scheme
 * (w_matrix = AMF_W_LOWER) on a grid with an axis-1 level above 10. */
amf_status amf_plan_create(const amf_problem* probs, int32_t n_probs, const amf_grid_spec* grid,
                           const amf_scheme* scheme, amf_precision precision, int32_t n_steps,
                           int32_t richardson, amf_plan** out);

/* Sizes and offsets of a plan. */
amf_status amf_plan_info_get(const amf_plan* plan, amf_plan_info* out);

/* Host metadata of one unit: problem index, levels (d entries), combination coefficient and the
 * element offset of the unit in every grid vector.  Any pointer may be NULL. */
amf_status amf_unit_info(const amf_plan* plan, int64_t unit, int32_t* problem, int32_t* levels,
                         double* coef, int64_t* offset);

/* Bind caller-owned device memory (>= workspace_bytes, 256-byte aligned) and upload the plan's
 * tables on `stream` (the call synchronises the stream before returning).  Rebinding is allowed
 * and invalidates the state. */
amf_status amf_plan_bind(amf_plan* plan, void* d_workspace, uint64_t bytes, void* stream);

/* Initial data (dis0): Y = payoff at every inner node of every unit; resets the step counter. */
amf_status amf_init(amf_plan* plan, void* stream);

/* Advance every unit by n AMFR-W steps (eq amfrw): per stage the explicit operator of Sketch 1,
 * the AMF chain of directional tridiagonal solves (Lemma lema:ls) along axes 1..d, the refinement
 * 2K - (I - theta dt F')K^(d) with F'K = F(K), a second chain, then Y += sum b_r K_r. */
amf_status amf_time_step(amf_plan* plan, int32_t n, void* stream);

/* amf_init + n_steps steps (and the 2*n_steps fine run when richardson = 1). */
amf_status amf_solve(amf_plan* plan, void* stream);

/* on = 1: amf_solve replays one hipGraph holding the whole solve (captured on the first call after
 * enabling, binding or changing the schedule; kernels only, no memset or copy nodes) instead of
 * launching ~10 d kernels per step from the host.  Not used while per-kernel profiling is on. */
amf_status amf_graph_enable(amf_plan* plan, int32_t on);

/* amf_combine, then wait for the stream and check the prices: AMF_E_NUMERIC (message naming the
 * first problem) when any price is not finite, the prices still written; AMF_OK otherwise.  For
 * callers that want the paper's failure signal of an unstable configuration without reading the
 * prices back themselves. */
amf_status amf_combine_checked(amf_plan* plan, double* d_prices, void* stream);

/* Per-unit value u_l(x_eval) by tensor-product linear interpolation (Section 5), in FP64, one per
 * unit in unit order, written to d_values (device, n_units doubles). */
amf_status amf_unit_values(amf_plan* plan, double* d_values, void* stream);

/* Prices: per problem, discount * sum_l c_l u_l(x_eval) in FP64 over its units in unit order
 * (eq modifiedCombTechnique), written to d_prices (device, n_problems doubles).  With Richardson,
 * the extrapolated price.  Asynchronous: non-finite prices (an unstable configuration) are written
 * as they are and are the caller's to detect. */
amf_status amf_combine(amf_plan* plan, double* d_prices, void* stream);

/* Copy the current solution Y (inner-node layout above, plan precision) to d_out (device, at least
 * vector_bytes).  The plan stores Y - g internally, g the payoff, which vanishes on the lower
 * faces; this call adds g back. */
amf_status amf_state_read(amf_plan* plan, void* d_out, void* stream);

/* Step-level entry points (parity testing of the individual steps).  d_in / d_out are grid vectors
 * in the inner-node layout and the plan precision, distinct from the workspace.
 *   amf_apply_operator: d_out = scale * F(d_in) of Sketch 1 on every unit; lower-face values are
 *     the payoff (increment = 0) or 0 (increment = 1).  d_in and d_out must not overlap.
 *   amf_axis_solve: solve (I - nu dt A_axis) d_out = d_in for every unit (Lemma lema:ls), with
 *     A_axis the directional second-difference matrix of (ffis) and nu, dt from the plan.
 *     d_out may equal d_in. */
amf_status amf_apply_operator(amf_plan* plan, const void* d_in, void* d_out, int32_t increment,
                              double scale, void* stream);
amf_status amf_axis_solve(amf_plan* plan, int32_t axis, const void* d_in, void* d_out, void* stream);

/* Launch schedule of a plan (tuning knobs).  Results agree across schedules up to rounding: the
 * operator's per-node arithmetic is the same in every schedule, but the fused axis-1 solve and the
 * unit-resident schedule order the tridiagonal recurrences differently from the streaming sweeps.
 *   stencil_nodes: consecutive axis-1 nodes evaluated per thread by the time-loop operator
 *                  (1, 2, 4 or 8; at most max_stencil_nodes = min(8, smallest M_1 of the plan)).
 *   xcd_remap:     assign each XCD a contiguous share of the blocks, so that blocks reading the
 *                  same halo planes share that XCD's L2: 1 = operator launches only, 2 = every
 *                  streaming launch (operators, sweeps, per-node kernels), 0 = off.
 *   resident:      1 = unit-resident schedule: one workgroup per component grid runs all time steps
 *                  of a call with the grid's vectors in LDS (only when resident_available, i.e.
 *                  every grid has at most 2048 points in FP32 or 1024 in FP64); 0 = streaming
 *                  schedule: one launch per operator / axis over all grids.
 *   fuse_axis0:    streaming schedule only: 1 = the time-loop operator launches also solve the
 *                  axis-1 systems of the first AMF factor (Lemma lema:ls) on the values they
 *                  produce.  Without march: no separate axis-1 sweep runs; allowed when
 *                  stencil_nodes >= 2, 256 * stencil_nodes >= the longest axis-1 line
 *                  (fuse_max_axis0 reports that line length) and that line has at most 1024
 *                  points.  With march: the grids whose axis-1 lines have at most 16 points are
 *                  solved in the operator launches, the others by the axis-1 sweep in place;
 *                  allowed when every axis-1 line has at most 1024 points.  0 = separate axis-1
 *                  sweep launches.
 *   march:         streaming schedule, d <= 4 only (march_available): 1 = the time-loop operators
 *                  run plane-tiled, one block per (grid, tile of the axes 1..d-1, range of V
 *                  planes) walking the V axis with the tile's neighbourhood in an LDS ring of
 *                  planes (every stencil neighbour read from LDS).
 * amf_schedule_set may be called at any time between enqueued calls; AMF_E_INVALID otherwise. */
typedef struct {
    uint32_t struct_size;
    int32_t stencil_nodes;
    int32_t xcd_remap;
    int32_t max_stencil_nodes;   /* read-only: filled by amf_schedule_get */
    int32_t resident;
    int32_t resident_available;  /* read-only: filled by amf_schedule_get */
    int32_t fuse_axis0;
    int32_t fuse_max_axis0;      /* read-only: longest axis-1 line M_1 of the plan */
    int32_t march;
    int32_t march_available;     /* read-only: filled by amf_schedule_get */
} amf_schedule;

amf_status amf_schedule_get(const amf_plan* plan, amf_schedule* out);
amf_status amf_schedule_set(amf_plan* plan, const amf_schedule* schedule);

/* Per-kernel timing (measurement support).  Between amf_profile_begin and amf_profile_end every
 * kernel the plan launches is bracketed by two HIP events recorded on its launch stream.
 * amf_profile_end waits for the last event and returns, per kernel class, the launch count, the
 * summed event time and the summed algorithmic bytes (bytes the kernel must move at minimum:
 * every vector it reads or writes once, in the plan precision). */
typedef enum {
    AMF_K_INIT = 0,             /* payoff / zero fills                                        */
    AMF_K_OPERATOR = 1,         /* Sketch-1 operator alone (F of the payoff; step-level API)  */
    AMF_K_STAGE1 = 2,           /* first-stage operator dt (F0(W) + F(g))                     */
    AMF_K_STAGE2 = 3,           /* second-stage operator dt (F0(W + a K1) + F(g)) + q K1      */
    AMF_K_REFINE = 4,           /* refinement 2 K - K^(d) + theta dt F(K^(d))                 */
    AMF_K_SWEEP_CONTIG = 5,     /* axis-1 solves, lines up to 16 points                       */
    AMF_K_SWEEP_CONTIG_LONG = 6,/* axis-1 solves, longer lines (partitioned, PCR over lanes)  */
    AMF_K_SWEEP_STRIDED = 7,    /* solves along axes 2..d, lines up to 16 points              */
    AMF_K_SWEEP_STRIDED_LONG = 8, /* ... longer lines                                         */
    AMF_K_SWEEP_UPDATE = 9,     /* last solve of a step fused with W += b1 K1 + b2 K2, short  */
    AMF_K_SWEEP_UPDATE_LONG = 10, /* ... longer lines                                         */
    AMF_K_UNIT_VALUES = 11,     /* interpolation at x_eval                                    */
    AMF_K_COMBINE = 12,         /* FP64 combination                                           */
    AMF_K_RESIDENT = 13,        /* unit-resident time loop (all stages and solves in LDS)     */
    AMF_K_LINCOMB = 14,         /* stage combinations sum_j c_j K_j of schemes with s > 2     */
    AMF_K_LOWER = 15,           /* (I - theta dt P) solves of the W = P method (wavefronts)   */
    AMF_K_COUNT = 16
} amf_kernel_class;

typedef struct {
    int32_t kernel;        /* amf_kernel_class */
    int32_t reserved;
    int64_t launches;
    double total_ms;
    double algo_bytes;
} amf_kernel_stat;

amf_status amf_profile_begin(amf_plan* plan);
/* stats: array of AMF_K_COUNT entries (one per class, in class order). */
amf_status amf_profile_end(amf_plan* plan, amf_kernel_stat* stats);

/* ------------------------------------------------------------------------------------------------
 * Pricing surrogate: a fully connected network n_in -> width (x depth, SiLU) -> 2 with BF16 weights
 * and activations and FP32 accumulation (gfx950 MFMA), trained on prices of the solver above.
 * Output 0 is the price, output 1 the logarithm of its estimated absolute error; callers route
 * requests whose estimated relative error exceeds their tolerance to the solver.  All shapes are
 * fixed at creation; device memory is caller-owned (one workspace, bound like a plan's). */
typedef struct amf_mlp amf_mlp;

typedef struct {
    int64_t n_params;                 /* FP32 master parameters (padded layout, see below)         */
    uint64_t workspace_bytes;
    int32_t n_in, width, depth, n_out, max_batch, layers;
    /* Parameter layout: per layer l a row-major weight block of layer_rows x layer_cols floats at
     * layer_w_offset, then layer_rows biases at layer_b_offset.  Rows and columns beyond the
     * logical sizes are zero padding and stay zero. */
    int32_t layer_rows[8], layer_cols[8];
    int64_t layer_w_offset[8], layer_b_offset[8];
} amf_mlp_info;

const char* amf_mlp_last_error(void);
/* n_in in [1, 32]; width a multiple of 32 in [32, 1024]; depth (hidden layers) in [1, 7]; n_out = 2;
 * weights drawn U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from `seed` (SplitMix64), biases 0. */
amf_status amf_mlp_create(int32_t n_in, int32_t width, int32_t depth, int32_t n_out, int32_t max_batch,
                          uint64_t seed, amf_mlp** out);
amf_status amf_mlp_info_get(const amf_mlp* mlp, amf_mlp_info* out);
/* Bind the workspace and upload the initial parameters (synchronises the stream). */
amf_status amf_mlp_bind(amf_mlp* mlp, void* d_workspace, uint64_t bytes, void* stream);
/* Host arrays: feature means and standard deviations (n_in each), target mean and scale (1 each).
 * out_log = 1: the network models log(price) (mean and scale of log prices; targets must be > 0),
 * so its residual is a relative error; out_log = 0: it models the price itself. */
amf_status amf_mlp_set_normalization(amf_mlp* mlp, const float* in_mean, const float* in_std,
                                     const float* out_mean, const float* out_std, int32_t out_log,
                                     void* stream);
/* direction 0: copy the FP32 master parameters to d_params; 1: load them from d_params (device). */
amf_status amf_mlp_params(amf_mlp* mlp, float* d_params, int32_t direction, void* stream);
/* Copy the gradient of the last backward pass / training step (same layout as the parameters). */
amf_status amf_mlp_grads(amf_mlp* mlp, float* d_grads, void* stream);
/* d_x: [batch, n_in] raw features (FP32, device).  d_out: [batch, 2] = (price, estimated relative
 * error of the price). */
amf_status amf_mlp_forward(amf_mlp* mlp, const float* d_x, int32_t batch, float* d_out, void* stream);
/* Inference only: the same outputs as amf_mlp_forward (same rounding points and accumulation order),
 * any batch >= 1, nothing kept for a backward pass.  Networks whose layers are at most 256 wide run
 * as one launch in which each workgroup takes 64 requests through every layer with the activations
 * in LDS; wider ones fall back to the training forward pass in chunks of max_batch. */
amf_status amf_mlp_infer(amf_mlp* mlp, const float* d_x, int32_t batch, float* d_out, void* stream);
/* After amf_mlp_forward of the same batch: gradient of sum_b dy[b] . y[b] with respect to the
 * parameters, y the two raw network outputs; d_dy is [batch, 2] FP32. */
amf_status amf_mlp_backward(amf_mlp* mlp, const float* d_dy, int32_t batch, void* stream);
/* One Adam step (beta 0.9/0.999, eps 1e-8) on the loss
 *   mean_b (y0 - t_b)^2 + err_weight (y1 - log(|y0 - t_b| + 1e-6))^2,  t_b the normalised target price;
 * the residual in the second term is held constant, t_b the normalised target (or log target).  d_loss (device, optional) receives the batch
 * sum before the division by the batch size. */
amf_status amf_mlp_train_step(amf_mlp* mlp, const float* d_x, const float* d_target, int32_t batch,
                              float lr, float err_weight, float* d_loss, void* stream);
void amf_mlp_destroy(amf_mlp* mlp);

/* Router of the surrogate (form 4): the box the network was trained on (n_in lower and upper
 * bounds, host arrays) and the calibration factor that scales its error estimate (Section "learned
 * part" of the build: the estimate is multiplied by calib before it is compared with a tolerance). */
amf_status amf_mlp_set_router(amf_mlp* mlp, const float* box_lo, const float* box_hi, float calib);

/* Price the n_problems requests of `fallback` with the network where it is trusted, else with the
 * solver.  d_x: [n, n_in] FP32 features on the device, row i describing problem i of the plan.
 * Request i is served by the network when its features lie inside the router's box, the network
 * price p_i is finite and its calibrated error estimate e_i = calib * est_i satisfies
 * e_i <= tol or e_i |p_i| <= abs_floor (a relative tolerance with an absolute floor); every other
 * request is routed to the solver: a plan of exactly those problems (same grid, scheme, precision,
 * steps and schedule) is built on the host, bound into the fallback plan's own workspace, solved
 * and combined (eq amfrw, eq modifiedCombTechnique).  Outputs (device): d_prices[n] FP64,
 * d_used_solver[n] 0/1.  Synchronises the stream.  When any request was routed, the fallback
 * plan's state is overwritten (its tables are uploaded again before returning): call amf_solve
 * before reading its state.  AMF_E_NUMERIC when a final price is not finite. */
amf_status amf_price_or_fallback(amf_mlp* mlp, amf_plan* fallback, const float* d_x, float tol,
                                 float abs_floor, double* d_prices, int32_t* d_used_solver, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): amf_solve + amf_combine of an UNBOUND (or bound) plan in
 * a library-owned workspace, a static device array of AMF_STATIC_WORKSPACE_BYTES per GPU that the
 * library holds until the process ends.  The call uploads the plan's tables into that array, runs
 * the whole solve eagerly (no graph) on `stream` and writes one FP64 price per problem to d_prices
 * (device).  It calls no hipMalloc/hipFree and no allocating library routine.  AMF_E_INVALID when
 * the plan needs more workspace than the array holds.  Every call on one GPU shares that GPU's
 * array and leaves its contents behind (nothing in it is assumed to start at zero): calls that
 * overlap on one GPU (two host threads, or two streams in flight) race and are not allowed.  A
 * plan bound with amf_plan_bind keeps its own workspace and state untouched.  The stream must
 * belong to the current device. */
#define AMF_STATIC_WORKSPACE_BYTES (64u << 20)
amf_status amf_solve_static(amf_plan* plan, double* d_prices, void* stream);

/* Release host resources.  Device memory stays owned by the caller.  NULL is allowed. */
void amf_plan_destroy(amf_plan* plan);

#ifdef __cplusplus
}
#endif
#endif /* AMFRW_H */
