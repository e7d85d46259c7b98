/* dgconv.h - C ABI of the MI355X upwind-DG convection library (libdgconv.so).
 *
 * The library computes the explicit upwind discontinuous-Galerkin convection operator and
 * its explicit Runge-Kutta substeps on affine simplicial meshes (triangles, tetrahedra):
 *
 *   C_h(u; w, z) = sum_T [ -int_T (w (x) u) : grad z dx + int_dT (u.n) w^ z ds ]   (Sec. 2.3)
 *   r            = -(M^V)^-1 C^V(u) w                                              (Sec. 2.4)
 *   ds w + (M^V)^-1 C^V(u) w = 0   integrated by SSP-RK3 substeps        (Sec. 3.2, propagation)
 *
 * w^ is the upwind value (pointwise, at the facet quadrature points), M^V the DG mass matrix,
 * diagonal for the orthonormal element basis (Sec. 2.3).  Where the paper's convecting
 * velocity is H(div)-conforming, a discontinuous convecting field here enters the facet term
 * through its averaged normal component beta = 1/2 (u^- + u^+) . n^-.
 *
 * Coefficient layout ("state"): [n_elem][dim][n_basis] row-major, element-major.  Component
 * i of element T is sum_m c[T][i][m] phi_m(F_T^-1 x) with phi_m the orthonormal Dubiner basis
 * on the unit reference simplex (order: total degree ascending, then the last index
 * descending, then the middle one) and F_T(xi) = v_0 + [v_1-v_0, ..., v_d-v_0] xi from the
 * element's vertex order as given, which the library never changes.
 *
 * Conventions for every call:
 *   - Return value: dg_status, 0 on success, negative on error; dg_last_error() gives a
 *     message for the calling thread.  No C++ exception crosses this boundary.
 *   - "dev" pointers are device memory on the current HIP device, 16-byte aligned, owned by
 *     the caller; "host" pointers are host memory owned by the caller.
 *   - stream is a hipStream_t passed as void* (NULL = the default stream).  Compute calls are
 *     asynchronous on that stream unless stated.
 *   - Input, output and work buffers of one call must not overlap unless stated.
 */
#ifndef DGCONV_H
#define DGCONV_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DG_OK = 0,
  DG_EINVAL = -1,       /* bad argument: null/misaligned pointer, size, k, dim, dt, n */
  DG_ENOMEM = -2,       /* device or host allocation failed */
  DG_EDEVICE = -3,      /* a HIP runtime call failed */
  DG_EUNSUPPORTED = -4, /* valid request this build does not implement (e.g. k too large) */
  DG_ENONFINITE = -5,   /* non-finite values detected */
  DG_EMESH = -6         /* degenerate element, unmatched or non-manifold facet */
} dg_status;

/* Arithmetic of the operator.  The state is FP64 except for DG_FP32 (FP32 state).  The
 * mixed variants keep the solution state, the facet flux, the lifted facet sums and the
 * Runge-Kutta stage updates in FP64 and run the basis contractions in lower precision. */
typedef enum {
  DG_FP64 = 0,      /* everything in FP64 */
  DG_FP32 = 1,      /* FP32 state and arithmetic */
  DG_MIX_F32 = 2,   /* FP64 state, flux, facet sums and RK; basis contractions (coefficients,
                       tables, volume sums) in FP32 on the vector units */
  DG_MIX_BF16x3 = 4,/* FP64 state, facet fluxes and RK; basis contractions as 3-way split
                       BF16 products on the matrix cores with FP32 accumulation */
  DG_MIX_F16x2 = 5  /* as above with 2-way split FP16 products (per-element power-of-two
                       scaling) */
  /* 3 (a 2-way BF16 split, 16 significant bits) is not provided: it cannot reach the 1e-6
     relative error the mixed variants are compared at */
} dg_precision;

typedef struct dg_mesh dg_mesh; /* opaque; immutable after creation */

typedef struct {
  int dim, k, n_basis;      /* n_basis = C(k+dim, dim) per component */
  int64_t n_elem, n_facet;  /* n_facet = (n_elem (dim+1) + n_bfacet) / 2 */
  int64_t n_dof;            /* n_elem * dim * n_basis */
  int nq_vol, nq_facet;     /* quadrature points per element volume / per facet (dg_volume_rule,
                               dg_facet_rule) */
  int n_types, n_tiles;     /* element classes with identical facet tables; 64-wide tiles */
  double h_min;             /* smallest facet measure (2D) or its square root (3D) */
  double volume;            /* sum of element volumes */
  int64_t n_bfacet;         /* boundary facets (0 on a fully periodic mesh) */
} dg_mesh_info;

/* Create a mesh of affine simplices (synchronous, host only).  The device tables are
 * uploaded to the current HIP device by the first compute call (dg_convection_apply,
 * dg_rk_substeps, dg_reduce), synchronously; later compute calls must run with the same
 * device current.  xyz: host [n_vert][dim]; elem: host [n_elem][dim+1] vertex ids, local
 * order = element frame; period: host [dim], per direction either a box length (> 0: facets
 * are matched by centroid modulo that period) or <= 0 for a bounded direction.  With every
 * direction periodic, every facet must be matched by a facet of another element; with a
 * bounded direction, facets left unmatched are boundary facets (Sec. 2.3: where the flow
 * enters, the upwind value comes from outside the domain), numbered in (element, local
 * facet) order, and the compute calls take their outer values (the _bc entry points).
 * k: 0..6 in 2D, 0..4 in 3D.
 * Errors: DG_EINVAL (dim not 2/3, k out of range, null pointers, vertex id out of range),
 * DG_EMESH (|det J| <= 1e-12 h^dim, unmatched facet on a fully periodic mesh, non-manifold
 * facet), DG_ENOMEM, DG_EDEVICE.  *out is set only on success; free with dg_mesh_destroy. */
dg_status dg_mesh_create(int dim, int k, int64_t n_vert, const double* xyz, int64_t n_elem,
                         const int64_t* elem, const double* period, dg_mesh** out);

/* Periodic unit box, n^dim squares split into 2 triangles or cubes split into 6 tetrahedra
 * (synchronous).  2D: square (i,j) -> lower (v00,v10,v11) id 2(jn+i), upper (v11,v01,v00)
 * id 2(jn+i)+1.  3D: cube (i,j,l), index (ln+j)n+i, Kuhn split along v000->v111: tet s =
 * (v000, v000+e_s0, v000+e_s0+e_s1, v111) for the permutations s of (x,y,z) in lexicographic
 * order, id 6*cube+index(s).  n >= 1. */
dg_status dg_mesh_create_box(int dim, int n, int k, dg_mesh** out);

void dg_mesh_destroy(dg_mesh* mesh); /* NULL is a no-op; synchronises the device */

dg_status dg_mesh_get_info(const dg_mesh* mesh, dg_mesh_info* out);

/* Unwrapped vertex coordinates of every element, host [n_elem][dim+1][dim] (synchronous). */
dg_status dg_mesh_get_vertices(const dg_mesh* mesh, double* xyz_out);

/* Facet connectivity, host [n_elem][dim+1] each: neighbour element across local facet f
 * (the facet opposite local vertex f) and that facet's local index in the neighbour.  On a
 * boundary facet b the neighbour entry is -1 - b and the facet index -1. */
dg_status dg_mesh_get_neighbors(const dg_mesh* mesh, int32_t* nbr_out, int32_t* nbr_facet_out);

/* L2 projection onto the DG space (synchronous, host).  dg_project_points writes the
 * physical points of a collapsed Gauss rule with n points per direction (n in 1..32),
 * host [n_elem][n^dim][dim]; dg_project takes a field sampled there, host
 * [n_elem][n^dim][dim], and writes the coefficients, host [n_elem][dim][n_basis]. */
dg_status dg_project_points(const dg_mesh* mesh, int n, double* xyz_out);
dg_status dg_project(const dg_mesh* mesh, int n, const double* vals, double* coef_out);

/* r = -(M^V)^-1 C^V(u) w  (one operator application).  Meshes with boundary facets need
 * dg_convection_apply_bc (DG_EINVAL here); the same holds for dg_rk_substeps, and
 * dg_rk_substeps_extrap and dg_richardson run on fully periodic meshes only
 * (DG_EUNSUPPORTED).
 * w: dev state; u: dev state (frozen convecting velocity) or NULL for u := w (the nonlinear
 * self-convection div(w (x) w)); r: dev state, output.  State element type is double except
 * for DG_FP32 (float).  r must not overlap w or u. */
dg_status dg_convection_apply(const dg_mesh* mesh, dg_precision prec, const void* w,
                              const void* u, void* r, void* stream);

/* Physical quadrature points of the boundary facets (host, synchronous): xyz_out host
 * [n_bfacet][nq_facet][dim], in boundary-facet order and, per facet, in the order of the
 * facet rule on the facet's vertices sorted lexicographically by coordinate (the order the
 * kernels use).  Outer values wb/ub are given at these points.  Nothing is written when the
 * mesh has no boundary facets (xyz_out may then be NULL). */
dg_status dg_boundary_points(const dg_mesh* mesh, double* xyz_out);

/* dg_convection_apply on a mesh with boundary facets (Sec. 2.3, upwind value from outside on
 * the inflow part of the boundary).  wb: dev [n_bfacet][nq_facet][dim], the outer values of
 * w at dg_boundary_points (same element type as w); ub: the outer values of the convecting
 * velocity there, required in frozen mode (u != NULL), ignored in self mode (u := w, so the
 * outer velocity is wb).  A boundary facet takes the interior flux formula with these outer
 * values: beta = 1/2 (u^- + u_b).n, F = beta {w} + |beta|/2 (w^- - w_b), so outflow facets
 * take w^- and inflow facets w_b.  On a mesh without boundary facets wb and ub may be NULL.
 * Errors as dg_convection_apply, plus DG_EINVAL for a missing wb or ub. */
dg_status dg_convection_apply_bc(const dg_mesh* mesh, dg_precision prec, const void* w,
                                 const void* u, const void* wb, const void* ub, void* r,
                                 void* stream);

/* n substeps of three-stage SSP-RK3 (Shu-Osher) with step dt for ds w = r(w), in place:
 *   w1 = w + dt r(w);  w2 = 3/4 w + 1/4 (w1 + dt r(w1));  w <- 1/3 w + 2/3 (w2 + dt r(w2)).
 * u: NULL (self-convection, re-evaluated at every stage) or a dev state (frozen velocity).
 * work: dev, at least 2 states, or NULL to use a buffer owned by the mesh (then concurrent
 * calls on one mesh must be serialised by the caller).  dt > 0 finite, n >= 0. */
dg_status dg_rk_substeps(const dg_mesh* mesh, dg_precision prec, void* w, double dt, int n,
                         const void* u, void* work, void* stream);

/* Pseudo-time (Richardson) iteration for the implicit convection problem of Sec. 3.3 with
 * frozen convection (eq. implconv):  v + tau (M^V)^-1 C^V(u) v = g.  Explicit Euler steps of
 * size ds in pseudo time (eq. implconvit, with the sign for which the fixed point solves
 * eq. implconv):
 *   res_i = g - v_i + tau r(v_i),  r(v) = -(M^V)^-1 C^V(u) v;   v_{i+1} = v_i + ds res_i,
 * stopping at the first i with ||res_i|| <= rtol ||res_0|| (L2 norm over the mesh), after at
 * most max_it updates.  Each update is one fused operator launch that also sums |det J| res^2
 * per tile; the criterion is evaluated on the device and the host checks it every few
 * iterations, so the iterates stop exactly at the first one that meets it.
 * v: dev FP64 state, the initial guess on entry (e.g. a copy of g), on exit the first iterate
 * meeting the criterion or v_max_it.  g, u: dev FP64 states (u is required: the convection is
 * frozen).  work: dev, at least one state, or NULL for the mesh-owned buffer (then calls on
 * one mesh must be serialised).  No argument may alias another.  prec: DG_FP64 or a mixed
 * precision (operator contractions only; the iterate, residual and norms stay FP64); DG_FP32
 * gives DG_EUNSUPPORTED.  tau finite, ds > 0, rtol >= 0, max_it >= 0.  iters_out (host, may
 * be NULL): the number n of updates (the returned iterate is v_n); res_out (host double[2],
 * may be NULL): ||res_0|| and the last residual norm evaluated.  Synchronises the stream. */
dg_status dg_richardson(const dg_mesh* mesh, dg_precision prec, double* v, const double* g,
                        const double* u, double tau, double ds, double rtol, int max_it,
                        double* work, void* stream, int* iters_out, double* res_out);

/* dg_rk_substeps on a mesh with boundary facets, the outer values wb, ub (as in
 * dg_convection_apply_bc) held fixed over the n substeps. */
dg_status dg_rk_substeps_bc(const dg_mesh* mesh, dg_precision prec, void* w, double dt, int n,
                            const void* u, const void* wb, const void* ub, void* work,
                            void* stream);

/* The propagation problem of Sec. 3.2 ("The propagation operator", eq. explproblem): n
 * SSP-RK3 substeps as dg_rk_substeps, with the convecting velocity extrapolated linearly in
 * time from two stored fields,
 *   u(s) = ua + (s - ta) / (tb - ta) (ub - ua),
 * evaluated at each stage's own time: substep j starts at s_j = t0 + j dt and its stages use
 * u(s_j), u(s_j + dt), u(s_j + dt/2).  ua, ub: dev states (same element type as w), neither
 * aliasing w; t0, ta, tb finite, tb != ta (ta, tb are the times of the stored fields, e.g. the
 * two previous steps for extrapolation).  Other arguments and errors as dg_rk_substeps. */
dg_status dg_rk_substeps_extrap(const dg_mesh* mesh, dg_precision prec, void* w, double dt,
                                int n, double t0, const void* ua, double ta, const void* ub,
                                double tb, void* work, void* stream);

/* Transfer between the H(div)-conforming velocity space W_h and the DG space V_h (Sec. 2.4,
 * eq. l2I; 2D meshes with 1 <= k <= 6, 3D meshes with 1 <= k <= 4).  W_h (Sec. 2.2:
 * element-wise [P^k]^d fields with continuous normal components) carries the
 * Brezzi-Douglas-Marini degrees of freedom:
 *   facet    int_F (v . n_F) q_l ds over an L2-orthonormal basis of P^k(F): n_F the outward
 *            normal of the lower-numbered element sharing F (of its element on a boundary
 *            facet); the facet parameter runs from its canonical vertices (lexicographic
 *            order), A + s (B - A) [+ t (C - A)]; 2D: q_l(s) = sqrt(2l+1) P_l(2s-1), l = 0..k;
 *            3D: q_l(s, t) = phi_l(s, t) / sqrt(2), phi_l the library's basis of the reference
 *            triangle (dg_eval_basis with dim 2), (k+1)(k+2)/2 functions;
 *   interior sign(det J) int_T v . (J^-T psi_r(F_T^-1 x)) dx, psi_r over the first-kind
 *            Nedelec space N_{k-1} of the reference simplex: e_i x^a y^b [z^c] for total
 *            degree <= k-2, then the rotations of the monomials m of degree k-2: (-y, x) m in
 *            2D, x ^ (e_i m) in 3D without i = 0 when x divides m; monomials by degree, a
 *            descending, then b descending, i ascending for each (k^2-1 functions in 2D,
 *            (k-1)(k+1)(k+2)/2 in 3D).
 * W_h coefficients u are the values of these functionals: the dofs of each facet (facets in
 * the order of their owner element, then local facet), then the interior dofs of each
 * element.  The numbering and device tables are built on the first transfer call
 * (synchronous).
 * dg_hdiv_info: *n_dof = dim W_h, *n_facet (may be NULL) = facets (host, synchronous).
 * dg_hdiv_reference: the reference dual basis, host [dim n_basis][dim][n_basis] (dof j in
 * local order: the facets' moments in each local facet's ascending-vertex parameter, then the
 * interior ones; then its DG coefficients on e_a phi_m of the reference simplex).
 * dg_transfer_to_dg: w_out = I u = (M^V)^-1 M^{U,V} u, the DG coefficients of the W_h field
 * (u: dev [n_dof] doubles; w_out: dev FP64 state).
 * dg_transfer_transpose: g_out = I^T f (f: dev FP64 state holding a functional's values on
 * the DG basis; g_out: dev [n_dof]); uses a mesh-owned work buffer, so calls on one mesh
 * must be serialised.  Errors: DG_EINVAL (dim, k, null pointers, aliasing). */
dg_status dg_hdiv_info(const dg_mesh* mesh, int64_t* n_dof, int64_t* n_facet);
dg_status dg_hdiv_reference(int dim, int k, double* table_out);
dg_status dg_transfer_to_dg(const dg_mesh* mesh, const double* u, double* w_out, void* stream);
dg_status dg_transfer_transpose(const dg_mesh* mesh, const double* f, double* g_out,
                                void* stream);

/* Reductions of FP64 states into out_dev (dev, doubles), deterministic (fixed summation
 * order, two passes over per-block partial results in a mesh-owned buffer):
 *   DG_RED_MAXVEL   out[0] = max of |a(x)| over the points of the collapsed Gauss-Jacobi rule
 *                   with ceil(3k/2)^dim points per element (the speed in the substep size)
 *   DG_RED_ENERGY   out[0] = 1/2 int |a|^2 dx, the kinetic energy whose stability the upwind
 *                   form gives (Sec. 2.3, eq. convstab; Sec. 2.5, the energy estimate of the
 *                   semidiscrete formulation)
 *   DG_RED_MOMENTUM out[0..dim-1] = int a dx (conserved by the single-valued upwind flux of
 *                   Sec. 2.3 on a periodic mesh)
 *   DG_RED_L2DIFF   out[0] = ||a - b||_L2, out[1] = ||b||_L2
 *   DG_RED_NONFINITE out[0] = number of non-finite coefficients of a
 * a, b: dev FP64 states (b only for DG_RED_L2DIFF); out_dev: dev, at least dim doubles.
 * Calls on one mesh share its partial-result buffer: concurrent calls on different streams
 * must be serialised by the caller.  Errors: DG_EINVAL (null pointer, unknown what, L2DIFF
 * without b). */
enum { DG_RED_MAXVEL = 0, DG_RED_ENERGY = 1, DG_RED_MOMENTUM = 2, DG_RED_L2DIFF = 3,
       DG_RED_NONFINITE = 4 };
dg_status dg_reduce(const dg_mesh* mesh, int what, const double* a, const double* b,
                    double* out_dev, void* stream);

/* dg_reduce for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same reductions, the same kernels and
 * the same results, with the per-block partial results in a static device array of the
 * library (768 KiB per device, held until the process ends) instead of the mesh's buffer.
 * No memory is allocated: the mesh's device tables must already be resident on the current
 * device (any earlier compute call there uploads them; DG_EINVAL otherwise).  Meshes of at
 * most 8 388 608 elements (DG_EINVAL above).  Every call on one device shares the array:
 * calls that overlap in time on one device (other streams, other threads, other meshes)
 * race and must be serialised by the caller.  Other arguments and errors as dg_reduce. */
dg_status dg_reduce_noalloc(const dg_mesh* mesh, int what, const double* a, const double* b,
                            double* out_dev, void* stream);

/* ---- Learned macro-step (2D, P3 elements): a per-element network replaces M substeps.
 * Network 80 -> 256 -> 256 -> 256 -> 20 with erf-GELU; BF16 matrix-core kernels with FP32
 * accumulation, FP32 master weights, Adam.  Flat FP32 parameters: W1 [256][80], b1 [256],
 * W2 [256][256], b2, W3 [256][256], b3, W4 [20][256], b4 [20] (layer: y = x W^T + b).
 * Input of element T: sigma_T / s [c_T, c_N0, c_N1, c_N2] (N_j across local facet j; each
 * block [dim][n_basis]); s = max |w| over the volume points, sigma_T = sign of the x
 * component of v1 - v0.  Output y_T is the remainder of the macro-step beyond forward Euler
 * over tau = M dt, in units of s^3 tau^2 / h (h = the mesh's h_min):
 *   w_T <- w_T + tau r(w)_T + sigma_T (s^3 tau^2 / h) y_T. */
typedef struct dg_surrogate dg_surrogate;

dg_status dg_surrogate_n_params(int64_t* n); /* 157460 */

/* Create a network for this mesh (allocates device memory; parameters zero until loaded).
 * M: substeps one macro-step replaces.  DG_EUNSUPPORTED unless dim = 2 and k = 3, and for a
 * mesh with boundary facets (the inputs need a neighbour across every facet); both checked
 * before any device work. */
dg_status dg_surrogate_create(const dg_mesh* mesh, int M, dg_surrogate** out);
void dg_surrogate_destroy(dg_surrogate* s);

/* FP32 master parameters from / to the host (synchronous); load resets the Adam state. */
dg_status dg_surrogate_load(dg_surrogate* s, const float* params_host, int64_t n);
dg_status dg_surrogate_save(const dg_surrogate* s, float* params_host, int64_t n);

/* Network inputs x_out (dev, FP32 [n][80]) and training targets t_out (dev, FP32 [n][20],
 * sigma_T h / (s^3 tau^2) (w1 - w0 - tau r0)_T with r0 = r(w0)) of the elements elems (dev
 * int32 [n], or NULL = all elements in order, then n = n_elem) of the FP64 states w, w0, w1,
 * r0; scale: dev double, s; tau > 0. */
dg_status dg_surrogate_features(const dg_surrogate* s, const double* w, const double* scale,
                                const int32_t* elems, int64_t n, float* x_out, void* stream);
dg_status dg_surrogate_targets(const dg_surrogate* s, const double* w0, const double* w1,
                               const double* r0, const double* scale, double tau,
                               const int32_t* elems, int64_t n, float* t_out, void* stream);

/* y = net(x): x dev FP32 [batch][80], y dev FP32 [batch][20] (inputs rounded to BF16). */
dg_status dg_surrogate_forward(dg_surrogate* s, const float* x, int64_t batch, float* y,
                               void* stream);
/* Mean-squared-error loss (dev float, may be NULL) and its gradient with respect to the
 * parameters (dev FP32 [157460], may be NULL) for inputs x and targets t (dev FP32). */
dg_status dg_surrogate_grad(dg_surrogate* s, const float* x, const float* t, int64_t batch,
                            float* grad_out, float* loss_dev, void* stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias correction) with learning rate lr. */
dg_status dg_surrogate_train_step(dg_surrogate* s, const float* x, const float* t,
                                  int64_t batch, float lr, float* loss_dev, void* stream);

/* One macro-step of M substeps of size dt on the FP64 state w (dev, in place, self-
 * convection; the propagation problem of Sec. 3.2 with u := w): candidate
 * w~ = w + tau r(w) + sigma (s^3 tau^2 / h) net(...), tau = M dt, accepted when its trapezoid
 * defect rho = ||w~ - w - (M dt / 2)(r(w) + r(w~))||_L2 / ||w~ - w||_L2 <= tol (a NaN defect,
 * from non-finite values, is never accepted; w~ = w gives 0 if r(w) + r(w~) = 0, else
 * infinity), else the M plain SSP-RK3 substeps are taken from w.  The check costs two
 * operator applications, less than one substep (three).
 * work: dev, at least 3 FP64 states (w~, r(w), r(w~); the fallback substeps reuse the last
 * two), or NULL for a buffer owned by s; it must not overlap w.  The network's batch buffers
 * are owned by s, so calls on one surrogate must be serialised.  Synchronises the stream
 * (the decision is made on the host); *accepted = 1 or 0, *rho_out = rho (may be NULL).
 * Errors: DG_EINVAL (null or misaligned pointers, dt <= 0 or non-finite, a surrogate created
 * for another mesh). */
dg_status dg_macro_step(const dg_mesh* mesh, dg_surrogate* s, double* w, double dt, double tol,
                        void* work, int* accepted, double* rho_out, void* stream);

/* Learned initial guess for dg_richardson (the pseudo-time problem of Sec. 3.3,
 * v + tau (M^V)^-1 C^V(u) v = g):
 *   v = g + tau r(g) + sigma_T (s^3 tau^2 / h) net(inputs of g),  r(g) = -(M^V)^-1 C^V(u) g,
 * s = max |g| over the volume points, inputs and sigma_T as for the macro-step.  The network
 * predicts the solution's remainder beyond one explicit Euler step of size tau; it is trained
 * with dg_surrogate_targets(w0 = g, w1 = the converged solution, r0 = r(g)).  g, v: dev FP64
 * states, v aliasing neither g nor u; u: dev FP64 frozen velocity, or NULL for u := g.
 * tau > 0 and finite.  Asynchronous on stream; uses workspace owned by s (calls on one
 * surrogate must be serialised).  DG_EINVAL for null or misaligned pointers or a surrogate
 * created for another mesh. */
dg_status dg_surrogate_warm_start(const dg_mesh* mesh, dg_surrogate* s, const double* g,
                                  const double* u, double tau, double* v, void* stream);

/* The library's reference basis on the unit simplex (host): vals [n_pts][n_basis] and,
 * if grads is not NULL, reference gradients [n_pts][n_basis][dim] at pts [n_pts][dim]. */
dg_status dg_eval_basis(int dim, int k, int64_t n_pts, const double* pts, double* vals,
                        double* grads);

/* The volume quadrature rule of the operator's volume term (Sec. 2.3, the cell integral of
 * C^V; its integrand has degree 3k-1, and the rule is exact to that degree, so it does not
 * change the operator): *n_out = number of points; if pts_out and wts_out are not NULL,
 * host pts_out [n][dim] in reference coordinates (= barycentric coordinates 1..dim) and
 * wts_out [n] summing to the reference simplex measure (1/2, 1/6).  A fully symmetric rule
 * with positive weights and interior points where the library has one (2D k 1..5,
 * 3D k 1..3), else the collapsed Gauss-Jacobi rule with ceil(3k/2)^dim points.  Host only.
 * Errors: DG_EINVAL (dim not 2/3, k < 0, n_out NULL), DG_EUNSUPPORTED (k above the compiled
 * range); *n_out is written only on success. */
dg_status dg_volume_rule(int dim, int k, int* n_out, double* pts_out, double* wts_out);

/* The facet quadrature rule of the operator's facet terms (Sec. 2.3, the facet integrals of
 * C^V with the upwind value taken pointwise, so the rule is part of the operator's
 * definition): exact to degree 3k; *n_out = number of points; if pts_out and wts_out are not
 * NULL, host pts_out [n][dim-1] (2D: s on the edge; 3D: (s, t), the point A + s (B - A) +
 * t (C - A) of the facet's canonically ordered vertices) and wts_out [n] summing to 1.  2D:
 * ceil((3k+1)/2) Gauss-Legendre points; 3D: the fully symmetric rule of degree 3k for k = 2
 * (12 points) and k = 3 (19 points), else the collapsed rule with ceil((3k+1)/2)^2 points.
 * Host only.  Errors: DG_EINVAL (dim not 2/3, k < 0, n_out NULL), DG_EUNSUPPORTED (k above
 * the compiled range); *n_out is written only on success. */
dg_status dg_facet_rule(int dim, int k, int* n_out, double* pts_out, double* wts_out);

const char* dg_last_error(void);
const char* dg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DGCONV_H */
