/*
 * lor.h -- C ABI of the MI355X LOR-Schwarz preconditioned conjugate gradient
 * library (Pazner, "Efficient low-order refined preconditioners for high-order
 * matrix-free continuous and discontinuous Galerkin methods").
 *
 * The library solves the high-order Poisson problem of Section 2,
 *     -div(grad u) = f in Omega,  u = 0 on the boundary        (eq. poisson)
 * discretized with continuous Galerkin (eq. fem / eq. system), symmetric
 * interior penalty DG (eq. ip) or BR2 DG (eq. br2) on Gauss-Lobatto (GLL)
 * tensor-product elements, by conjugate gradients preconditioned with the
 * overlapping vertex-patch additive Schwarz method of eq. as (eq. dg-as for
 * DG), whose patch solvers are element-structured multigrid V-cycles on the
 * low-order refined operator with MDF-ordered ILU(0) smoothing
 * (Sections 3.1-3.4).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * - Every function returns an int status: LOR_OK (0) or a negative LOR_E*
 *   code.  No function throws or aborts across the ABI.  lor_error_string()
 *   gives a static description.
 * - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *   memory of the current device (for example torch tensors' data_ptr()).
 *   The caller owns every buffer it passes; the library never frees them.
 * - "stream" is a hipStream_t passed as void*; NULL means the default stream.
 *   Work is enqueued on that stream; functions that return host results
 *   synchronise it.  A handle must be used by one stream at a time.
 * - Floating-point vectors are float64.
 *   CG vectors are "L-vectors": the GLL grid nodes of the whole mesh that are
 *   not on the Dirichlet boundary, in lexicographic order with x fastest
 *   (the grid has n_i*p+1 points in direction i).  With LOR_BC_NEUMANN every
 *   grid node is an unknown.
 *   DG vectors are "E-vectors": element-major (elements lexicographic, x
 *   fastest), (p+1)^d nodes per element (lexicographic, x fastest).
 */
#ifndef LOR_H
#define LOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LOR_OK          0
#define LOR_EINVAL     -1  /* bad argument, NaN/Inf in an input              */
#define LOR_EJACOBIAN  -2  /* element map with det J <= 0 at a GLL node      */
#define LOR_EPIVOT     -3  /* IC(0) pivot <= 0 or not finite                  */
#define LOR_EBREAKDOWN -4  /* p^T A p <= 0 or r^T z <= 0 in CG               */
#define LOR_ENOCONV    -5  /* maxit reached; x and info hold the last iterate */
#define LOR_EHIP       -6  /* HIP runtime error                               */
#define LOR_ENOMEM     -7  /* workspace missing or too small                  */
#define LOR_ESTATE     -8  /* call not valid in the handle's current state    */
#define LOR_EACCURACY  -9  /* the recursive residual reached rtol but the true
                              residual ||b - A x|| stays above it after
                              residual replacement: rtol lies below the
                              accuracy float64 attains for this operator
                              (x and info hold the best iterate)           */

typedef struct lor_handle lor_handle_t;   /* opaque, owned by the library */

typedef enum { LOR_CG = 0, LOR_IP = 1, LOR_BR2 = 2 } lor_method_t;
typedef enum { LOR_BC_DIRICHLET = 0, LOR_BC_NEUMANN = 1 } lor_bc_t;

/* Structured block of quads (dim 2) or hexes (dim 3) covering a domain; each
 * element is the image of [0,1]^d under the Q1 map of its 2^d vertices
 * (Section 2).  vertex_xyz: HOST, (n0+1)(n1+1)(n2+1) x dim float64, vertices
 * lexicographic with x fastest; copied during lor_setup. */
typedef struct {
  int dim;                  /* 2 or 3 */
  int n[3];                 /* elements per direction (n[2] ignored in 2D) */
  const double *vertex_xyz; /* host */
  int bc;                   /* lor_bc_t; Neumann only supports lor_apply_A */
  /* Coefficient b of -div(b grad u) = f (Section 4.2), HOST, NULL for b = 1:
   * b at every element's GLL nodes, n_el x (p+1)^d float64, elements and
   * local nodes lexicographic (x fastest) -- the layout of a DG E-vector, so
   * that b may jump across element faces.  b >= 0, not zero everywhere;
   * CG only.  It multiplies the quadrature weight of each node in the
   * high-order operator, and each LOR sub-element's Q1 stiffness is scaled
   * by the mean of b over the sub-element's 2^d corners (GLL nodes of the
   * element holding it).  Copied during lor_setup. */
  const double *coef;
  /* Curved (isoparametric) elements, HOST, NULL for straight ones: the
   * coordinates of every GLL grid node for the degree p of lor_setup,
   * (n0 p+1)(n1 p+1)(n2 p+1) x dim float64, x fastest.  Element e is then
   * the image of [0,1]^d under the degree-p interpolant of its own nodes
   * (the geometric factors come from the derivatives of that interpolant at
   * the GLL nodes), and the LOR sub-elements have these nodes as corners.
   * vertex_xyz must hold the same points at the vertices (the nodes with
   * every index a multiple of p).  CG only.  Copied during lor_setup. */
  const double *node_xyz;
} lor_mesh_t;

#define LOR_PREC_FP64   0   /* every step in float64 */
#define LOR_PREC_MIXED  1   /* preconditioner applied in float32 */

/* Elimination order of the IC(0) smoother on every patch level (Section 3.4
 * compares MDF with reverse Cuthill-McKee and approximate minimum degree and
 * finds MDF and RCM comparable). */
#define LOR_ORD_MDF     0   /* minimum discarded fill (Section 3.4)           */
#define LOR_ORD_NATURAL 1   /* patch-local lexicographic                      */
#define LOR_ORD_RCM     2   /* reverse Cuthill-McKee on the stencil graph of
                               the patch box: start at a node of minimum
                               degree (smallest index), neighbours in
                               increasing degree (ties by index), reversed   */

/* Weights of the patch corrections in the Schwarz sum. */
#define LOR_PROLONG_SUM 0   /* eq. as: corrections added unweighted           */
#define LOR_PROLONG_POU 1   /* each correction scaled by 1/c(i), c(i) the
                               number of patches holding unknown i (the
                               counting-matrix weighting of Section 4.1; a
                               partition of unity, not symmetric: flexible CG
                               is used)                                      */

/* Subdomains of the Schwarz preconditioner. */
#define LOR_PATCH_VERTEX 0  /* one patch per mesh vertex plus the coarse
                               space (eq. as, Section 3.2)                    */
#define LOR_PATCH_SINGLE 1  /* B(1) of Section 4.1: a single patch, the whole
                               domain: one V-cycle of the LOR hierarchy with
                               IC(0) smoothing (in the chosen order) on every
                               level and the exact solve on the last level,
                               the original mesh T_p (its interior vertices,
                               at most 40000, by a dense inverse); no separate
                               coarse space.  The sweeps follow the dependency
                               levels of the elimination order over the whole
                               domain, so they are far longer than a patch's */
#define LOR_PATCH_SLABS  2  /* B(n) of Section 4.5: nslabs overlapping
                               subdomains, slabs of elements along x (bounds
                               i n[0] / nslabs, widened by one element on
                               their inner sides), each solved like B(1) on
                               its part of the hierarchy; no coarse space    */
#define LOR_PATCH_VERTEX_ISO 3 /* vertex patches enlarged for isotropic overlap
                               (Section 4.5): from each vertex the patch grows,
                               per direction and sense, one element at a time
                               until the vertex reached is at least 0.9 times
                               the longest mesh edge at the vertex away (or
                               the boundary is reached); each solved like B(1)
                               on its box, plus the coarse space of eq. as.
                               The box-patch modes (SINGLE, SLABS, VERTEX_ISO)
                               run in float64.  A box whose dependency levels
                               have at most sweep_grid_rows rows (and whose
                               finest level at most 65536) runs its whole
                               V-cycle in one workgroup, every such box in
                               one launch; larger boxes take one launch per
                               sweep segment and transfer, on four streams.
                               The corrections are added to z one colour of
                               boxes (disjoint level-0 boxes) at a time, in a
                               fixed order: B r is bit-reproducible          */

typedef struct {
  int precision;       /* LOR_PREC_*                                        */
  int ordering;        /* LOR_ORD_*                                         */
  int flexible;        /* 0: PCG, 1: flexible CG FCG(1); forced on for MIXED
                          and for LOR_PROLONG_POU                           */
  int nthreads;        /* host threads for the ordering pass; 0 = all cores */
  int prolong_weights; /* LOR_PROLONG_*                                     */
  int patch_mode;      /* LOR_PATCH_*                                       */
  int sweep_grid_rows; /* box-patch modes: a dependency level with more rows
                          than this is swept by a launch over the whole
                          device, runs of smaller levels by one workgroup
                          (a barrier between levels); a box with no such
                          level runs its whole V-cycle in one workgroup;
                          0 = 512                                       */
  int nslabs;          /* LOR_PATCH_SLABS: number of subdomains, 1..n[0]    */
  int deterministic;   /* 1: the vertex patches' corrections are added
                          without atomics, one vertex-parity class of
                          patches (disjoint boxes) per launch, classes in a
                          fixed order: B r is bit-reproducible (and so is
                          the whole solve where the operator is: 3D with
                          4 <= p <= 7), at about four times the patch
                          kernel's time.  The box-patch modes are always
                          bit-reproducible.  No patch network then.         */
  int launch_order;    /* LOR_LAUNCH_*: the order in which the vertex-patch
                          kernel's workgroups take the patches            */
  int operator_geometry; /* LOR_GEOM_*                                      */
  int nn_fallback;     /* with a patch network attached (lor_nn_attach):
                          1 (default) = lor_pcg_solve leaves the network for
                          the patch V-cycles, restarting flexible CG from
                          the current iterate's true residual, when the
                          iteration breaks down or stalls (the recursive
                          residual falls less than 2x over 16 iterations);
                          0 = the network to the end                     */
} lor_options_t;

/* Geometric factors of the operator.  LOR_GEOM_STORED (default): computed
 * once at set-up and streamed by every application (48 bytes per element
 * node).  LOR_GEOM_ONFLY: in 3D CG with straight elements, b = 1 and
 * 4 <= p <= 7 the operator recomputes G = w|J| J^-1 J^-T at every node from
 * the element's vertices instead, and G is not stored (ignored otherwise):
 * less memory, but measured slower (16^3, p = 6: 33 us against 23 us for
 * the element kernel; equal at 32^3), as the kernel is not bound by the
 * stream of G. */
#define LOR_GEOM_STORED 0
#define LOR_GEOM_ONFLY  1

/* Launch order of the vertex-patch kernel.  LOR_LAUNCH_AUTO (the default)
 * times both orders at set-up (a few launches on the handle's workspace)
 * and keeps the faster; lor_launch_order reports the choice. */
#define LOR_LAUNCH_AUTO    0
#define LOR_LAUNCH_VERTEX  1  /* vertex order                                  */
#define LOR_LAUNCH_BUCKETS 2  /* patches by decreasing work (rows over all
                                 smoothed levels), vertex order among equals:
                                 interior, face, edge and corner patches, so
                                 the largest start first and the smallest fill
                                 the launch's last round                      */

typedef struct {
  int    iters;        /* CG iterations performed (all restarts together)  */
  int    status;       /* LOR_OK, LOR_ENOCONV, LOR_EACCURACY, LOR_EBREAKDOWN */
  double rel_res;      /* ||r_k||_2 / ||b||_2 of the recursive residual    */
  double rel_res_true; /* ||b - A x||_2 / ||b||_2 recomputed at exit       */
  double t_solve;      /* seconds, measured with HIP events                */
  double t_setup;      /* seconds lor_setup took for this handle (host clock) */
  int    replacements; /* residual replacements (restarts from b - A x)    */
  int    fallback_iter; /* iteration at which a network-preconditioned solve
                           switched to the patch V-cycles (nn_fallback);
                           -1 if it did not                                */
} lor_solve_info_t;

/* Fill *opt with the defaults (FP64, MDF, PCG, all cores). */
int lor_default_options(lor_options_t *opt);

const char *lor_error_string(int code);

/* Detail of the last LOR_EHIP failure on the calling thread (which HIP call
 * and its error string) or of a set-up LOR_EINVAL that has a reason (patch
 * too large for the LDS); empty if none.  Static thread-local storage. */
const char *lor_last_error_detail(void);

/* Set up the discretization and the preconditioner (Sections 2 and 3).
 * p: polynomial degree, 1 <= p <= 14.  method: lor_method_t.
 * penalty: eta > 0, ignored for CG; IP uses sigma = eta p^2 / h_e on each
 *   face (eq. ip, h_e = min |K|/|e| over the elements at the face, volumes
 *   and areas by GLL quadrature); BR2 uses eta as the factor of the lifting
 *   term (eq. br2), which with the collocated GLL element mass is a
 *   node-wise penalty sigma_q = eta c^2 sum_K omega_q / (w|J|)_q^K on the
 *   face nodes (c = 1/2 inside, 1 on the boundary).  DG boundary conditions
 *   are imposed weakly through the boundary faces (Dirichlet) or not at all
 *   (Neumann: no boundary faces).
 *   In 3D a patch's V-cycle vectors live in the 160 KiB LDS of one CU
 *   (2 (2p-1)^3 + (2 s_1 - 1)^3 values, s_1 the sub-intervals of level 1),
 *   which limits p to 11 with LOR_PREC_FP64 and to 13 with LOR_PREC_MIXED;
 *   a larger p returns LOR_EINVAL with the reason in lor_last_error_detail.
 * opt: NULL for defaults.  stream: used for the device part of the set-up.
 * Allocates the device data the handle needs (geometric factors, LOR
 * stencils, patch factors, coarse inverse) and builds everything.
 * Errors: LOR_EINVAL (bad sizes, NaN vertex), LOR_EJACOBIAN, LOR_EPIVOT,
 * LOR_EHIP.  On error *out is NULL and nothing is leaked. */
int lor_setup(const lor_mesh_t *mesh, int p, int method, double penalty,
              const lor_options_t *opt, void *stream, lor_handle_t **out);

/* The launch order the handle uses (LOR_LAUNCH_VERTEX or _BUCKETS) and,
 * after an autotuned set-up, the measured milliseconds per patch launch in
 * each order (0 otherwise); either pointer may be NULL. */
int lor_launch_order(const lor_handle_t *h, int *order, double *ms_vertex, double *ms_buckets);

/* Number of unknowns: the L-vector length for CG, n_el (p+1)^d for DG. */
int lor_ndofs(const lor_handle_t *h, int64_t *n);

/* Bytes of device memory the library holds for the handle (after
 * lor_bind_workspace only the cached workspaces of batched solves). */
int lor_device_bytes(const lor_handle_t *h, size_t *bytes);

/* Caller-owned device memory (section 8 of the boundary: the caller's
 * allocator, e.g. torch's, owns the device memory).  lor_setup builds the
 * handle's device data (geometric factors, LOR stencils, patch factors,
 * coarse inverse, solve workspace) in library allocations;
 * lor_workspace_bytes gives their total size (each rounded up to 256 bytes),
 * and lor_bind_workspace moves all of it into the caller's DEVICE buffer
 * dev_ptr (256-byte aligned, at least that many bytes) on `stream`, then
 * frees the library's copies.  Afterwards the buffer must outlive the
 * handle, must not be touched by the caller, and lor_free leaves it alone.
 * Results are unchanged.  Errors: LOR_EINVAL (NULL or misaligned pointer),
 * LOR_ENOMEM (buffer too small; needed size in lor_last_error_detail),
 * LOR_ESTATE (already bound).  Once bound, lor_workspace_bytes returns the
 * bound size. */
int lor_workspace_bytes(const lor_handle_t *h, size_t *bytes);
int lor_bind_workspace(lor_handle_t *h, void *dev_ptr, size_t bytes, void *stream);

/* Coordinates of the unknowns, HOST output of ndofs x dim float64.  CG: the
 * GLL grid node evaluated with the map of element min(g_i / p, n_i - 1) in
 * each direction.  DG: each element's own map at its GLL nodes. */
int lor_dof_coords(const lor_handle_t *h, double *host_xyz);

/* Coordinates of every element's GLL nodes (each element's own map, or its
 * own nodes on a curved mesh), HOST
 * output of n_el (p+1)^d x dim float64 in the E-vector layout: where a
 * variable coefficient is evaluated (lor_mesh_t.coef).  Uses a temporary
 * device buffer. */
int lor_element_coords(const lor_handle_t *h, double *host_xyz);

/* b = M_p f with the collocated GLL mass (eq. system right-hand side):
 * b_i = sum over elements containing node i of w_i |J_i| f_i.
 * f_dev: DEVICE, f at the unknowns (same layout as b); b_dev: DEVICE out. */
int lor_assemble_rhs(lor_handle_t *h, const double *f_dev, double *b_dev, void *stream);

/* y = A x, matrix-free by sum factorization (Section 2; eq. ip / eq. br2
 * for DG).  x_dev, y_dev: DEVICE, ndofs float64, must not alias. */
int lor_apply_A(lor_handle_t *h, const double *x_dev, double *y_dev, void *stream);

/* z = B r: additive Schwarz preconditioner of eq. as.  DG (eq. dg-as):
 * z = D_B^-1 r on the element-boundary nodes (point Jacobi of A_DG on V_B)
 * plus E B E^T r with E the injection of the conforming space.
 * r_dev, z_dev: DEVICE, ndofs float64, must not alias.  LOR_ESTATE for a
 * Neumann handle (no preconditioner). */
int lor_apply_P(lor_handle_t *h, const double *r_dev, double *z_dev, void *stream);

/* z_i = B_i r_i for n problems (eq. as / eq. dg-as for each), the patch
 * corrections of up to four problems in one launch: consecutive handles
 * with vertex patches whose corrections use atomics (not deterministic, no
 * patch network) and of the same dimension and precision share a launch;
 * any other handle is applied alone, as by lor_apply_P.  hs: n distinct
 * handles (each holds one workspace); r[i], z[i]: DEVICE, ndofs(hs[i])
 * float64 each, r[i] != z[i].  Same results as n calls of lor_apply_P up
 * to the order of the atomic additions.  LOR_EINVAL for a repeated or null
 * handle or vector, LOR_ESTATE for a handle without a preconditioner. */
int lor_apply_P_batch(lor_handle_t *const *hs, int n, const double *const *r, double *const *z,
                      void *stream);

/* z = B r exactly as lor_apply_P computes it, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the call allocates, frees and memsets
 * nothing and records no events.  Its scratch vectors (the coarse-space
 * residual and correction, n_c values each, and for DG the conforming
 * residual and correction, one conforming L-vector each) live in a static
 * device array of 8 MiB per GPU, held until the process ends; a handle that
 * needs more returns LOR_ENOMEM (reason in lor_last_error_detail).  Every
 * call on one GPU shares that array: calls that overlap on one GPU (other
 * streams or threads) race.  The handle's device must be current.
 * r_dev, z_dev: DEVICE, ndofs float64, must not alias.  LOR_ESTATE for a
 * handle without preconditioner or with a patch network attached. */
int lor_apply_P_noalloc(lor_handle_t *h, const double *r_dev, double *z_dev, void *stream);

/* Scratch bytes lor_apply_P_noalloc needs for h, and the static capacity. */
int lor_noalloc_scratch_bytes(const lor_handle_t *h, size_t *needed, size_t *capacity);

/* Solve A x = b by preconditioned (or flexible) CG (Section 4) from x = 0
 * until ||r_k||_2 <= rtol ||b||_2 (recursive residual) or maxit iterations.
 * When the recursive residual meets rtol, the true residual b - A x is
 * computed; if it is above rtol ||b||_2 the iteration restarts from it
 * (residual replacement: r = b - A x, z = B r, p = z) while the true
 * residual keeps falling by at least 4x per restart, at most 4 times.
 * b_dev: DEVICE in; x_dev: DEVICE out.  info: HOST out, may be NULL.
 * Returns LOR_OK (true residual <= rtol ||b||_2), LOR_ENOCONV (maxit
 * reached; x holds the last iterate), LOR_EACCURACY (true residual stuck
 * above rtol) or LOR_EBREAKDOWN. */
int lor_pcg_solve(lor_handle_t *h, const double *b_dev, double *x_dev,
                  double rtol, int maxit, lor_solve_info_t *info, void *stream);

/* Batched solve of many independent problems and right-hand sides:
 * pair k = i * nrhs + j solves A_i x_k = b_k with handle hs[i] (i < nprob,
 * j < nrhs), exactly as lor_pcg_solve would (same kernels in the same
 * order; the patch corrections, and the operator outside 5 <= p+1 <= 8 in 3D,
 * are accumulated with float64 atomics, so the last bits of any two solves
 * may differ).  Every pair gets its own device
 * workspace.  The CG iterations are captured once into HIP graphs (8
 * iterations per graph, kernels turn into no-ops after a pair's device-side
 * convergence flag is set), replayed on four worker streams until every
 * pair has converged or reached maxit, so that small problems run
 * concurrently and launch costs are paid once per chunk.  Where the
 * preconditioner allows it (vertex patches with atomics, no patch
 * network), a graph runs up to four right-hand sides of a problem in
 * lockstep with one patch launch per iteration for all of them; with more
 * such groups than streams, groups too small to fill the device with their
 * patch launch share graphs, up to four problems of the same dimension and
 * precision per patch launch.
 * A handle must not be used by another call during the batch (it may
 * appear several times in hs).
 * b, x: HOST arrays of nprob*nrhs DEVICE pointers (ndofs of the pair's
 * handle each); stream: the caller's stream, ordered before and after the
 * batch.  info: HOST array of nprob*nrhs entries (may be NULL); t_solve is
 * the time of the whole batch from the moment workspaces and graphs are
 * ready.  Returns LOR_OK or the first failing pair's status (LOR_ENOCONV,
 * LOR_EACCURACY, LOR_EBREAKDOWN, LOR_EINVAL); LOR_ESTATE for a handle
 * without preconditioner.  Residual replacement as in lor_pcg_solve.  The
 * pairs' workspaces are allocated the first time a handle serves that many
 * pairs in one call and kept on the handle for later batches (counted by
 * lor_device_bytes, released by lor_free); graphs are captured per call. */
int lor_pcg_solve_batch(lor_handle_t *const *hs, int nprob, int nrhs, const double *const *b_dev,
                        double *const *x_dev, double rtol, int maxit, lor_solve_info_t *info,
                        void *stream);

/* ---------------------------------------------------------------------
 * Learned patch correction.  A small 3D convolutional network (3 layers of
 * 3x3x3 convolutions, `channels` hidden channels, ReLU) acts on one vertex
 * patch at a time, on the level-0 patch grid of G = 2p-1 points per
 * direction (grid point g_d is level-0 node v_d p - p + 1 + g_d).  Input
 * channels: the patch residual divided by its 2-norm s_j, and the mask of
 * the patch unknowns; output: an approximation of the patch V-cycle
 * (Section 3.3) of the normalised residual.  Trained on pairs (residual,
 * V-cycle) that the method generates; in LOR_NN_REPLACE mode the
 * preconditioner becomes z = coarse correction + sum_j R_j^T s_j
 * net(R_j r / s_j) (eq. as with the network in place of the patch solves);
 * flexible CG is required (the network is nonlinear).  3D CG handles only.
 * Arithmetic: BF16 MFMA products with float32 accumulation, float32 master
 * weights and Adam moments.
 * Parameters (HOST float64 vectors of lor_nn_param_count values): layer by
 * layer W [27 cin][cout] row-major (row k cin + c, kernel offset
 * k = (dx+1) + 3 (dy+1) + 9 (dz+1)), then the bias [cout]; cin = 2, C, C and
 * cout = C, C, 1.
 * Data: X [nb][G^3][2] (float32, residual / s_j and mask), T [nb][G^3]
 * (float32 targets), both DEVICE.  A network must not be used by two calls
 * at once; a handle with an attached network is refused by
 * lor_pcg_solve_batch. */
typedef struct lor_nn lor_nn_t;
#define LOR_NN_OFF       0   /* patch V-cycles (eq. as) */
#define LOR_NN_REPLACE   1   /* the network stands in for every patch V-cycle */
#define LOR_NN_WARMSTART 2   /* y_j = s_j net(r_j / s_j) starts the patch solve:
                                z_j = y_j + V_j(r_j - A_j y_j), A_j the patch's
                                level-0 LOR matrix (a V-cycle-corrected guess) */

int lor_nn_param_count(int channels, int64_t *count);
/* channels: multiple of 16, 16..64.  max_batch: patches per network pass
 * (sizes the device buffers: about 4.5 (G^3 max_batch) (27 channels) bytes). */
int lor_nn_create(lor_handle_t *h, int channels, const double *params_host, int max_batch,
                  void *stream, lor_nn_t **out);
int lor_nn_get_params(const lor_nn_t *nn, double *params_host);
/* Number of patches J (vertex order) and grid points per direction G. */
int lor_nn_shape(const lor_nn_t *nn, int *npatch, int *grid);
/* Training data for the global residual r_dev (ndofs): X [J][G^3][2],
 * T [J][G^3] and scale [J] (DEVICE outputs), from the handle's own patch
 * V-cycles. */
int lor_nn_patch_data(lor_nn_t *nn, const double *r_dev, float *X_dev, float *T_dev,
                      double *scale_dev, void *stream);
/* Y [nb][G^3] = network output (masked), nb <= max_batch. */
int lor_nn_forward(lor_nn_t *nn, const float *X_dev, int nb, float *Y_dev, void *stream);
/* Masked mean squared error of the batch and its gradient (HOST outputs,
 * the parameter layout), without an update. */
int lor_nn_gradients(lor_nn_t *nn, const float *X_dev, const float *T_dev, int nb, double *loss,
                     double *grad_host, void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the batch; *loss is
 * the loss before the step. */
int lor_nn_train_step(lor_nn_t *nn, const float *X_dev, const float *T_dev, int nb, double lr,
                      double *loss, void *stream);
/* Use nn in h's preconditioner (LOR_NN_REPLACE or LOR_NN_WARMSTART) or not
 * (LOR_NN_OFF, nn may be NULL).  The network must have been created for h.
 * LOR_NN_REPLACE needs LOR_PROLONG_SUM, and either mode vertex patches
 * without `deterministic` (LOR_ESTATE otherwise).
 * Either mode makes the preconditioner nonlinear: lor_pcg_solve then runs
 * flexible CG.  The first warm-start attach allocates the predictions of
 * every patch, J (2p-1)^3 floats and J doubles (LOR_ENOMEM on failure). */
int lor_nn_attach(lor_handle_t *h, lor_nn_t *nn, int mode);
int lor_nn_free(lor_nn_t *nn);
/* The network's BF16 matrix product, exposed for tests: C[M][ldc] (float32,
 * DEVICE) = A B with A(i,k) = A[i ai + k ak], B(k,j) = B[k bk + j bj]
 * (bfloat16 bit patterns, DEVICE); M, N, K multiples of 16. */
int lor_bf16_gemm(int M, int N, int K, const uint16_t *A, int64_t ai, int64_t ak,
                  const uint16_t *B, int64_t bk, int64_t bj, float *C, int64_t ldc, void *stream);
/* The float64 matrix-core product of the coarse inverse's set-up (the
 * rank-b updates of blocked Gauss-Jordan elimination, Section 3.2), exposed
 * for tests: C = alpha A B + beta C, row major, A(i,k) = A[i lda + k],
 * B(k,j) = B[k ldb + j], C(i,j) = C[i ldc + j], all DEVICE, any m, n, k >= 0
 * (lda >= k, ldb >= n, ldc >= n); with beta == 0 C is not read.  Enqueued on
 * the stream (no synchronization).  LOR_EINVAL for bad sizes or pointers. */
int lor_f64_gemm(int m, int n, int k, double alpha, const double *A, int64_t lda, const double *B,
                 int64_t ldb, double beta, double *C, int64_t ldc, void *stream);

/* Integer maps for parity checks, HOST output.  If host_out is NULL only
 * *len is set.  which:
 *   LOR_MAP_LDOF          L-vector index -> flat GLL grid index
 *   LOR_MAP_ORDER         MDF orders of every (patch, level) concatenated,
 *                         patches in vertex order, levels fine to coarse
 *                         (the coarsest level, solved exactly, has none)
 *   LOR_MAP_ORDER_OFFSET  start of each (patch, level) in LOR_MAP_ORDER,
 *                         J*(L-1)+1 entries
 *   LOR_MAP_SCHEDULE      dependency-level starts of each (patch, level)
 *                         sweep, concatenated (depth+1 entries each)
 *   LOR_MAP_SCHEDULE_OFFSET start of each (patch, level) in LOR_MAP_SCHEDULE
 *   LOR_MAP_E2L           DG only: E-vector node -> conforming L-vector index
 *                         of the same GLL grid node, -1 on the Dirichlet
 *                         boundary (the injection E of eq. dg-as)
 * LOR_MAP_LDOF and the Schwarz maps refer to the conforming L-vector for DG
 * too (the space the DG preconditioner's Schwarz part works in). */
#define LOR_MAP_LDOF             0
#define LOR_MAP_ORDER            1
#define LOR_MAP_ORDER_OFFSET     2
#define LOR_MAP_SCHEDULE         3
#define LOR_MAP_SCHEDULE_OFFSET  4
#define LOR_MAP_E2L              5
int lor_export_maps(const lor_handle_t *h, int which, int32_t *host_out, int64_t *len);

/* Assembled LOR stencils of level k of the global element-structured
 * hierarchy (Section 3.3), HOST output: (3^d) x npts float64, slot-major;
 * slot = sum_i (o_i + 1) 3^i for the grid offset o in {-1,0,1}^d, points
 * lexicographic (x fastest) over the level grid, boundary points included.
 * If host_out is NULL only *len is set.  Returns LOR_EINVAL for a bad k. */
int lor_export_stencils(const lor_handle_t *h, int level, double *host_out, int64_t *len);

/* Per-kernel timing with HIP events recorded on the calling stream around
 * every launch of the hot kernels (for roofline measurements).
 * lor_timing(h, 1) clears the record and starts recording, lor_timing(h, 0)
 * stops.  lor_timing_read returns the summed duration (ms) and the number of
 * launches of one kernel class since the last reset; it synchronises the
 * recorded events.  which: */
#define LOR_T_APPLY_A   0   /* sum-factorized operator kernel            */
#define LOR_T_PATCH     1   /* patch V-cycle kernel (all patches)        */
#define LOR_T_COARSE    2   /* coarse restrict + inverse GEMV + prolong  */
int lor_timing(lor_handle_t *h, int enable);
int lor_timing_read(const lor_handle_t *h, int which, double *total_ms, int64_t *count);

/* ---- host-only utilities (no device needed): the set-up building blocks,
 * exposed so that their integer results can be checked bit for bit. ---- */

/* GLL nodes x[0..p] and weights w[0..p] on [0,1] (Section 3.1), correctly
 * rounded to float64.  HOST outputs of p+1 doubles. 1 <= p <= 14. */
int lor_gll(int p, double *x, double *w);

/* Ordering and IC(0) factor of one patch matrix (Section 3.4).
 * dim: 2 or 3; m: box extents (dim entries, each >= 1); rows: HOST,
 * n x 3^dim float64 stencil rows of the box points (n = prod m, x fastest;
 * slot as in lor_export_stencils; couplings leaving the box are ignored).
 * ordering: LOR_ORD_MDF, LOR_ORD_NATURAL (index order) or LOR_ORD_RCM.
 * HOST outputs (any may be NULL): order[n] elimination order;
 * level_ptr[n+1] dependency-level starts of the forward sweep, *depth levels;
 * L[n x 3^dim] (row i: l_im at earlier neighbours m, l_mi at later ones);
 * D[n] pivots.  Returns LOR_EPIVOT for a pivot <= 0. */
int lor_mdf_order(int dim, const int *m, const double *rows, int ordering, int32_t *order,
                  int32_t *level_ptr, int32_t *depth, double *L, double *D);

/* Release every resource of the handle (NULL is accepted). */
int lor_free(lor_handle_t *h);

#ifdef __cplusplus
}
#endif
#endif /* LOR_H */
