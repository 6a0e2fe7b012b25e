/*
 * frmi.h -- C ABI of the MI355X-native Flux Reconstruction right-hand side.
 *
 * The library evaluates the FR right-hand side of the paper's Sec. "Flux
 * Reconstruction" (conservation law eq:gov, mapped to reference elements via the
 * transformed equation, then the four steps eq:disu, eq:comm_flux, second
 * eq:disu and eq:FRfinal) for the compressible Euler and Navier--Stokes
 * equations on periodic meshes of hexahedra (orders 1..4, Gauss--Legendre
 * points; straight, with metric terms formed from the corners, or curved, with
 * metric terms stored per point as in Sec. "Curved elements") and tetrahedra
 * (order 4, the alpha-optimised points of Fig. mesh; straight, or curved with
 * metric terms stored per solution point), or of pyramids with affine bases (order
 * 4, Sec. "Mixed elements and domain decomposition"; meshes of pyramids only),
 * advances it with classical
 * RK4 ("a suitable explicit time integration scheme") or with an adaptive
 * embedded pair (Sec. "Adaptive time stepping"), and applies the entropy-bounded
 * modal filter of Sec. "Numerical Stability" with an optional learned warm start
 * of its per-element search.
 * All device work runs in hand-written HIP kernels for gfx950.
 *
 * Conventions
 *   Pointers named *_dev are device pointers (e.g. from hipMalloc or a PyTorch
 *   CUDA tensor); the others are host pointers.  Host arrays are read during the
 *   call only.  Device arrays are owned by the caller and must stay valid until
 *   the context's stream has completed the work that uses them.
 *   Every call enqueues on the stream given at setup and returns without
 *   synchronising unless stated.  Device faults surface as FR_ERR_DEVICE at the
 *   next synchronising call.  No C++ exception crosses this interface.
 *   fr_last_error(ctx) returns a message for the last failing call on ctx, or
 *   for the calling thread when ctx is NULL (e.g. after a failed setup).
 *
 * Canonical state layout (used by fr_pack / fr_unpack and for initial conditions)
 *   FP64, per element type block (hexahedra first, then tetrahedra; pyramids alone), elements in
 *   the order they appear in the mesh, [elem][var][sol_pt] with var = (rho, rho u,
 *   rho v, rho w, E).  Hex solution point zeta = i + (p+1)(j + (p+1)k), i along the
 *   first reference axis, Gauss--Legendre nodes increasing.  Tet solution points
 *   in the printed order of Fig. mesh(c).  Pyramid solution points: 5 layers at
 *   the Gauss--Legendre z nodes (increasing), layer k the (5-k) x (5-k)
 *   Gauss--Legendre grid scaled by s = (1 - z)/2, x fastest (55 points).
 * Native layout (what fr_rhs / fr_rk_step / fr_filter operate on)
 *   Internal: per type block [sol_pt][var][E_pad] (element fastest), elements in
 *   the native order (see fr_params.elem_order).  Sizes come from fr_layout; do
 *   not rely on them beyond allocation.
 */
#ifndef FRMI_H
#define FRMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fr_ctx_s* fr_ctx;

typedef enum {
  FR_OK = 0,
  FR_ERR_ARG = 1,          /* bad argument (NULL, size, value out of range)          */
  FR_ERR_MESH = 2,         /* unpaired face, non-conforming flux points, J <= 0     */
  FR_ERR_ALLOC = 3,        /* device or host allocation failed                       */
  FR_ERR_DEVICE = 4,       /* a HIP call or kernel failed                            */
  FR_ERR_NONFINITE = 5,    /* fr_check found a NaN/Inf or a non-positive rho or p    */
  FR_ERR_STATE = 6,        /* call not valid in the context's current state          */
  FR_ERR_UNSUPPORTED = 7   /* order / element type / option not supported            */
} fr_status;

enum { FR_EULER = 0, FR_NAVIER_STOKES = 1 };
enum { FR_RUSANOV = 0, FR_HLLC = 1 };
enum { FR_FP64 = 0, FR_FP32 = 1, FR_FP32_BF16X3 = 2 };
enum { FR_HEX = 0, FR_TET = 1, FR_PYR = 2 };
enum { FR_METRIC_CONSERVATIVE = 0, FR_METRIC_CROSS = 1 };

/* Solver parameters.  struct_size must be sizeof(fr_params). */
typedef struct {
  uint32_t struct_size;
  int32_t system;          /* FR_EULER or FR_NAVIER_STOKES                           */
  int32_t order;           /* hexahedra: 1..4; tetrahedra need 4                     */
  int32_t riemann;         /* FR_RUSANOV or FR_HLLC (common flux of eq:comm_flux)    */
  int32_t precision;       /* FR_FP64, or FR_FP32: FP32 kernels on deviation
                              variables du = u - u_ref (FP64 RK accumulation), or
                              FR_FP32_BF16X3: as FR_FP32 with the dense tetrahedral
                              operator products done as BF16x3 split products
                              (hi*hi + hi*lo + lo*hi, FP32 accumulation on the bf16
                              matrix cores); the hexahedra of a mixed mesh run the
                              FP32 form (their 1-D line contractions have no dense
                              product to split); FR_ERR_UNSUPPORTED for a mesh
                              without tetrahedra                                     */
  int32_t elem_order;      /* native element order of each type block: 1 keeps the
                              input order, 2 renumbers along a Morton curve of the
                              element centroids (face neighbours share tiles and
                              cache lines), 0 (default) takes whichever of the two
                              spreads the face neighbours of a 64-element tile over
                              fewer tiles.  Canonical arrays always follow the input
                              order.                                                 */
  double gamma;            /* ratio of specific heats                                */
  double mu;               /* constant dynamic viscosity (Navier--Stokes)           */
  double prandtl;          /* Prandtl number                                         */
  double ldg_beta;         /* LDG switch, relative to each face's left side         */
  double ldg_tau;          /* LDG penalty                                            */
  double u_ref[5];         /* reference state of the FP32 deviation form             */
  double filt_eps_rho;     /* entropy filter: density floor                          */
  double filt_eps_p;       /* entropy filter: pressure floor                         */
  double filt_eps_s;       /* entropy filter: relative entropy tolerance (all >= 0)  */
  double filt_zeta_max_coef; /* zeta_max = coef * p^2, coef > 0 and finite          */
  int32_t filt_bits;       /* dyadic search depth n (2^n grid), 1..30                */
  int32_t hex_metric;      /* metric terms of curved elements (fr_setup_mesh_curved,
                              fr_setup_mesh_curved_tet; the name predates the latter):
                              FR_METRIC_CONSERVATIVE (default) or FR_METRIC_CROSS     */
} fr_params;

typedef struct {
  int32_t n_types;         /* 1 or 2                                                  */
  int32_t etype[2];        /* FR_HEX / FR_TET / FR_PYR of each block                 */
  int64_t n_elem[2];       /* elements per block                                     */
  int64_t e_pad[2];        /* padded element count of the native layout             */
  int32_t n_sp[2];         /* solution points per element                            */
  int32_t n_fp[2];         /* flux points per element                                */
  int64_t canon_offset[2]; /* offset (in values) of each block in the canonical array*/
  int64_t native_offset[2];/* offset (in values) of each block in the native array   */
  int64_t canon_len;       /* total values of the canonical array                    */
  int64_t native_len;      /* total values of a native state                          */
  int32_t native_dtype;    /* FR_FP64 or FR_FP32 (native state values of fr_rhs)     */
  int32_t reserved;
} fr_layout_t;

typedef struct {
  int64_t n_troubled;      /* elements with the filter active (k != 0)               */
  int64_t n_fallback;      /* elements filtered at zeta_max because no k satisfied   */
  int64_t n_evals;         /* constraint evaluations over troubled elements          */
  double  seconds;         /* device time of the call                                */
  int64_t n_candidates;    /* elements the detection passed to the exact search      */
} fr_filter_stats;

/* Adaptive time stepping (Sec. "Adaptive time stepping": low-storage Runge--Kutta with
 * an embedded pair; the error estimate of each step, normalised, decides acceptance and
 * the next step size).  Scheme: the third-order, four-stage pair with a second-order
 * embedded solution RK3(2)4[2R+]C of Kennedy, Carpenter & Lewis (2000), carried in the
 * two-register "2R+" form plus an error register.  Norm: RMS over all values of
 * e / (atol + rtol max(|u_n|, |u_{n+1}|)), e = u_{n+1} - u^_{n+1}; accepted if <= 1;
 * next step dt min(fac_max, max(fac_min, safety norm^(-1/3))) (fac_min if the norm is
 * not finite); the last step is shortened to land on t_end. */
typedef struct {
  double atol, rtol;       /* error scale per value: atol + rtol max(|u_n|, |u_{n+1}|) (> 0) */
  double safety;           /* controller safety factor (0, 1]                         */
  double fac_min, fac_max; /* bounds of the step-size change, 0 < fac_min <= 1 <= fac_max */
  int32_t max_attempts;    /* accepted + rejected steps before returning (>= 1)       */
  int32_t reserved;
} fr_adaptive_params;

typedef struct {
  int64_t accepted, rejected;  /* steps                                               */
  int64_t n_rhs;               /* right-hand sides evaluated (4 per attempted step)   */
  double t;                    /* time reached (t_end unless max_attempts ran out)    */
  double dt_next;              /* proposed size of the next step                      */
  double last_norm;            /* error norm of the last attempted step               */
} fr_adaptive_stats;

/* Fill p with defaults: Euler, order 3, Rusanov, FP64, gamma 1.4, mu 1/1600,
 * Pr 0.71, beta 0.5, tau 0.1, u_ref = (1, 0, 0, 0, 1/((gamma-1) gamma Ma^2) with
 * Ma 0.1), filter floors 1e-8, entropy tolerance 1e-4, zeta_max 40 p^2, 20 bits. */
void fr_default_params(fr_params* p);

/* Build a context for a periodic conforming mesh (Sec. "Flux Reconstruction":
 * conforming tessellation, mapping, Jacobians).
 *   xyz      [n_vert][3] vertex coordinates.
 *   period   [3] box lengths; faces are matched by centroids modulo these and
 *            flux points by coordinates after removing the face's periodic shift.
 *            A zero entry means "not periodic in that direction".
 *   etype    [n_elem] FR_HEX (8-node, VTK corner order) or FR_TET (4-node, corners
 *            in the order (-1,-1,-1) (1,-1,-1) (-1,-1,1) (-1,1,-1) of the reference), or
 *            FR_PYR (5-node: the base corners in cyclic order, then the apex, as the
 *            reference (-1,-1,-1) (1,-1,-1) (1,1,-1) (-1,1,-1) (0,0,1); Sec. "Mixed
 *            elements and domain decomposition": pyramids with an affine base, so the
 *            base must be a parallelogram, corner 2 = corner 1 + corner 3 - corner 0,
 *            else FR_ERR_MESH).  Pyramids are order 4 (55 solution points of the
 *            rational pyramid space, layered Gauss--Legendre; 85 flux points: the base's
 *            5 x 5 Gauss--Legendre grid and each triangle the 15 face points of the
 *            p = 4 tetrahedron; DG lifting) and come in meshes of pyramids only: a mesh
 *            mixing them with other types is FR_ERR_UNSUPPORTED, as are the entropy
 *            filter, the MLP calls and FR_FP32_BF16X3 on such a context.
 *   enodes   [n_elem][8] corner indices (tets use the first 4, pyramids 5).
 *   stream   hipStream_t for all work of the context (NULL = default stream).
 * Synchronous.  Errors: FR_ERR_ARG, FR_ERR_MESH, FR_ERR_UNSUPPORTED, FR_ERR_ALLOC. */
fr_status fr_setup_mesh(const fr_params* p, int64_t n_vert, const double* xyz,
                        const double* period, int64_t n_elem, const int32_t* etype,
                        const int64_t* enodes, void* stream, fr_ctx* out);

/* Build a context for a periodic conforming mesh of curved hexahedra (Sec. "Curved
 * elements": metric terms kept per point of curved elements).
 *   geo_order  q in 1..min(4, order): geometry order of every element.
 *   ho_nodes   [n_elem][(q+1)^3] indices into xyz, tensor order: node i + (q+1)(j + (q+1)k)
 *              sits at reference point (-1 + 2i/q, -1 + 2j/q, -1 + 2k/q) of the map
 *              x(xi) = sum_n N_n(xi) x_n (tensor Lagrange polynomials on those points).
 *              Faces are matched from the 8 corner nodes as in fr_setup_mesh; elements
 *              sharing a face must share its nodes (conforming curved faces).
 *   p->hex_metric  FR_METRIC_CONSERVATIVE: S = J G^{-1} as the curl of the order-p
 *              Gauss--Lobatto interpolant of x_l grad x_m ((n, m, l) cyclic,
 *              S_rn = -[curl V^(n)]_r): divergence-free at the solution points, so a
 *              uniform stream stays uniform, and equal and opposite normals on every
 *              shared face (periodic ones too, which is why q <= order); x_l is taken
 *              relative to the element's node 0 (no change in exact arithmetic for
 *              q <= order, no cancellation of the coordinates' size against h^2);
 *              FR_METRIC_CROSS: S from the exact Jacobian at every point.
 *              J is det(dx/dxi) of the exact map in both cases.
 * The metric terms are stored per point (9 + 1 per solution point, 3 per flux point) in
 * the kernels' arithmetic type instead of being derived from 24 corner coefficients;
 * every other call behaves as for fr_setup_mesh.  Synchronous.
 * Errors: FR_ERR_ARG (NULL, index out of range), FR_ERR_UNSUPPORTED (q outside
 * 1..min(4, order)), FR_ERR_MESH (unpaired face, J <= 0 at a solution or flux point),
 * FR_ERR_ALLOC. */
fr_status fr_setup_mesh_curved(const fr_params* p, int32_t geo_order, int64_t n_vert, const double* xyz,
                               const double* period, int64_t n_elem, const int64_t* ho_nodes, void* stream,
                               fr_ctx* out);

/* Build a context for a periodic conforming mesh of curved tetrahedra (Sec. "Curved
 * elements", the tetrahedra of Fig. fsp), solution order 4 (p->order must be 4).
 *   geo_order  q in 1..4: geometry order of every element.
 *   ho_nodes   [n_elem][(q+1)(q+2)(q+3)/6] indices into xyz: the nodes (i, j, k) with
 *              i + j + k <= q, k outermost, then j, then i, at reference point
 *              (-1 + 2i/q, -1 + 2j/q, -1 + 2k/q) of the reference tetrahedron with
 *              corners (-1,-1,-1) (1,-1,-1) (-1,-1,1) (-1,1,-1); the map is their
 *              Lagrange interpolant of total degree q.  Faces are matched from the 4
 *              corner nodes as in fr_setup_mesh; elements sharing a face must share its
 *              nodes.
 *   p->hex_metric  FR_METRIC_CONSERVATIVE: the curl form as for hexahedra with the
 *              interpolant of total degree 4 on the 35 solution points (15 on each
 *              face, so the two elements of a face agree on its unit normal);
 *              FR_METRIC_CROSS: S from the exact Jacobian, a polynomial of degree
 *              2(q - 1), which the solution polynomials miss for q = 4.  J is
 *              det(dx/dxi) of the exact map in both cases.
 * The metric terms are stored per solution point (9 + 1 values) and, per flux point, the
 * scaled normal S^T n~ of its face at the collocated solution point (3 values), in the
 * kernels' arithmetic type; every other call behaves as for fr_setup_mesh.  Synchronous.
 * Errors: FR_ERR_ARG (NULL, index out of range), FR_ERR_UNSUPPORTED (q outside 1..4,
 * order other than 4), FR_ERR_MESH (unpaired face, J <= 0 at a solution point),
 * FR_ERR_ALLOC. */
fr_status fr_setup_mesh_curved_tet(const fr_params* p, int32_t geo_order, int64_t n_vert, const double* xyz,
                                   const double* period, int64_t n_elem, const int64_t* ho_nodes, void* stream,
                                   fr_ctx* out);

fr_status fr_layout(fr_ctx ctx, fr_layout_t* out);

/* Physical solution points, canonical order: [canon_len / 5][3] (host).  Synchronous. */
fr_status fr_sol_points(fr_ctx ctx, double* xyz);

/* Canonical FP64 state (device) -> native state (device), and back.  In the FP32
 * form the native state holds du = u - u_ref in FP32. */
fr_status fr_pack(fr_ctx ctx, const double* canon_dev, void* native_dev);
fr_status fr_unpack(fr_ctx ctx, const void* native_dev, double* canon_dev);

/* Canonical FP64 state (device) <-> FP64 native state (device): the layout of the
 * state that fr_rk_step, fr_filter and fr_check work on, in both precisions. */
fr_status fr_pack64(fr_ctx ctx, const double* canon_dev, double* native_dev);
fr_status fr_unpack64(fr_ctx ctx, const double* native_dev, double* canon_dev);

/* A native right-hand side (fr_rhs output, native dtype) -> canonical FP64 values
 * (no reference state is added in the FP32 form: R is not a deviation). */
fr_status fr_unpack_rhs(fr_ctx ctx, const void* r_dev, double* canon_dev);

/* r = du/dt of the FR scheme (steps 1-4 of Sec. "Flux Reconstruction", with
 * R = -(div f~)/J from the transformed equation).  Native layout; dtype as
 * fr_layout().native_dtype.  u and r must not alias. */
fr_status fr_rhs(fr_ctx ctx, const void* u_dev, void* r_dev);

/* n_steps classical RK4 steps of size dt on the FP64 native state u (in place).
 * filter_mode: -1 no filter; 0 plain entropy filter; 1 MLP warm-started filter.
 * The filter is applied to every stage state and to the new state, with the
 * entropy bound taken from the state at the start of the step.  In the FP32 form
 * the right-hand sides run on FP32 deviations while the stage states, the
 * accumulation and the filter (with its checks) stay FP64.  Both element types
 * (the filter treats each block with its own modal basis). */
fr_status fr_rk_step(fr_ctx ctx, void* u_dev, double dt, int32_t n_steps, int32_t filter_mode);

/* Defaults of fr_rk_adaptive: atol = rtol = 1e-6, safety 0.9, fac_min 0.3, fac_max 2.5,
 * 100000 attempts. */
void fr_default_adaptive_params(fr_adaptive_params* p);

/* Advance the FP64 native state u (in place) from t = 0 to t_end with adaptive steps
 * of the embedded pair above, starting from the step size dt0; rejected steps restore
 * u_n.  In the FP32 form the right-hand sides run on FP32 deviations while the state,
 * the stage registers' FP64 parts, the error register and the norm are FP64.  No
 * entropy filter.  stats (host) receives the counts; the call synchronises once per
 * attempted step (the norm decides on the host).  Errors: FR_ERR_ARG (NULL, t_end or
 * dt0 not positive and finite, parameters out of range), FR_ERR_ALLOC, FR_ERR_DEVICE;
 * a non-finite norm counts as a rejected step (the controller shrinks dt). */
fr_status fr_rk_adaptive(fr_ctx ctx, void* u_dev, double t_end, double dt0, const fr_adaptive_params* prm,
                         fr_adaptive_stats* stats);

/* Entropy-bounded modal filter (Sec. "Numerical Stability", entropy filtering)
 * of the FP64 native state u in place; the minimum entropy of each element's
 * neighbourhood is taken from u_prev (may equal u).  mode 0 plain bisection,
 * 1 MLP warm start (weights must be set).  k_dev (device, [sum n_elem] int32,
 * canonical element order, or NULL) receives the dyadic strength index
 * (0 untouched, -1 fallback).  stats (host, or NULL) synchronises.
 * Modes: tensor Legendre (hexahedra, exponent (i^2 + j^2 + k^2) / p^2) or the
 * orthonormal basis graded by total degree d (tetrahedra, exponent (d / p)^2).
 * Check points: solution and flux points (on the tetrahedra the flux points
 * coincide with solution points). */
fr_status fr_filter(fr_ctx ctx, void* u_dev, const void* u_prev_dev, int32_t mode,
                    int32_t* k_dev, fr_filter_stats* stats);

/* MLP warm start (16 -> 64 -> 64 -> 1, tanh).  Flat FP32 parameters (5,313):
 * W1[64][16] b1[64] W2[64][64] b2[64] w3[64] b3[1]; inputs standardised with
 * x_mean[16], x_std[16].  Host pointers; set/get synchronise. */
fr_status fr_mlp_set_weights(fr_ctx ctx, const float* w, const float* x_mean, const float* x_std);
fr_status fr_mlp_get_weights(fr_ctx ctx, float* w);

/* Features of the troubled elements of u (neighbourhood entropy from u_prev):
 * x_dev [cap][16] FP32 raw (unstandardised) features, elem_dev [cap] canonical
 * element ids, k_dev [cap] the plain filter's dyadic index for each (training
 * target).  *n (host) receives the count (synchronises); at most cap written. */
fr_status fr_mlp_features(fr_ctx ctx, const void* u_dev, const void* u_prev_dev,
                          float* x_dev, int32_t* elem_dev, int32_t* k_dev, int64_t cap, int64_t* n);

/* Training data from the plain filter: n_steps filtered RK4 steps of size dt on
 * the FP64 native state u (in place, plain filter on every stage state and the new
 * state); at every filter application the raw features (x_dev [cap][16]) and the
 * plain search's dyadic index (k_dev [cap], -1 = fallback) of each element that
 * fails the checks are recorded before it is filtered.  *n (host) receives the
 * number of rows written (at most cap).  Synchronises after every filter call. */
fr_status fr_mlp_collect(fr_ctx ctx, void* u_dev, double dt, int32_t n_steps, float* x_dev, int32_t* k_dev,
                         int64_t cap, int64_t* n);

/* Predictions y_dev [n] for raw features x_dev [n][16] with the current weights. */
fr_status fr_mlp_forward(fr_ctx ctx, const float* x_dev, int64_t n, float* y_dev);

/* Mean-squared-error loss and its gradient for a batch: x_dev [n][16] raw
 * features, y_dev [n] targets; grad_dev [5313], loss_dev [1] (device).         */
fr_status fr_mlp_grad(fr_ctx ctx, const float* x_dev, const float* y_dev, int64_t n,
                      float* grad_dev, float* loss_dev);

/* For callers that cannot allocate device memory during the call (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): fr_mlp_grad without any
 * allocation.  Same arguments, kernels and result as fr_mlp_grad (x_dev [n][16] raw
 * features, y_dev [n] targets, grad_dev [5313] and loss_dev [1] device outputs), but the
 * per-sample forward/backward quantities live in a fixed device array of the library
 * (FR_MLP_STATIC_MAX_BATCH x 274 floats, about 4.5 MB per GPU, held until the process
 * ends) instead of context workspace grown on demand.  Every call on a GPU shares that
 * GPU's array, so calls that overlap on one GPU (other streams, other contexts, other
 * threads) race; each call writes every entry it later reads, so nothing carries over
 * between calls.  Errors: FR_ERR_ARG (NULL, n outside 1..FR_MLP_STATIC_MAX_BATCH),
 * FR_ERR_STATE (weights not set), FR_ERR_DEVICE (the array's address could not be taken
 * at setup, or a launch failed). */
#define FR_MLP_STATIC_MAX_BATCH 4096
fr_status fr_mlp_grad_static(fr_ctx ctx, const float* x_dev, const float* y_dev, int64_t n,
                             float* grad_dev, float* loss_dev);

/* Adam training on (x, y) pairs (device): n_steps minibatches of `batch` drawn by
 * the host-side permutation perm_dev [n_steps * batch] (int32 row ids).  lr,
 * beta1, beta2, eps as in Adam.  loss_hist_dev [n_steps] (device, or NULL).   */
fr_status fr_mlp_train(fr_ctx ctx, const float* x_dev, const float* y_dev, int64_t n,
                       const int32_t* perm_dev, int32_t n_steps, int32_t batch,
                       float lr, float beta1, float beta2, float eps, float* loss_hist_dev);

/* Scan an FP64 native state for NaN/Inf or rho <= 0 or p <= 0 at solution points.
 * Synchronises; FR_ERR_NONFINITE if any is found. */
fr_status fr_check(fr_ctx ctx, const void* u_dev);

/* Per-kernel device timing with HIP events recorded around every kernel launch
 * of the context on its stream (adds a little launch overhead; off by default).
 * fr_profile(ctx, 1) clears and enables, fr_profile(ctx, 0) disables.
 * fr_profile_read synchronises and fills up to cap records (host). */
typedef struct {
  char name[48];           /* kernel family, e.g. "hex_div_ns_p3"                    */
  int64_t launches;
  double total_ms;         /* summed event-measured device time                      */
} fr_kernel_time;
fr_status fr_profile(fr_ctx ctx, int32_t enable);
fr_status fr_profile_read(fr_ctx ctx, fr_kernel_time* out, int32_t cap, int32_t* n);

fr_status fr_sync(fr_ctx ctx);
void fr_destroy(fr_ctx ctx);
const char* fr_last_error(fr_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* FRMI_H */
