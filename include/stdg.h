/*
 * stdg.h - C ABI of the MI355X staggered space-time DG pressure library.
 *
 * The library implements the hot path of the staggered semi-implicit
 * space-time discontinuous Galerkin scheme of Tavelli & Dumbser
 * (arXiv 1601.07384) on tetrahedral meshes:
 *   - the pressure Schur operator of eq. CS_19 (Sec. 2.4), applied matrix-free,
 *   - its Krylov solve (CG for p_gamma = 0, GMRES otherwise; Sec. 2.7 and
 *     Sec. 3.2 use the same unpreconditioned solvers), in FP64 or as an
 *     FP32-inner / FP64-refinement solve,
 *   - one Picard pressure-correction time step (Sec. 2.6, steps 0-6).
 *
 * Conventions shared by every entry point
 *   - Status: every function returns an int; 0 = STDG_OK, > 0 a soft
 *     outcome, < 0 an error.  A thread-local message for the last error is
 *     returned by stdg_last_error().  No C++ exception crosses the ABI.
 *   - Element order: the library renumbers elements along a Hilbert
 *     space-filling curve (unless stdg_config.reorder = 0).  Every device
 *     vector below is in this internal order; stdg_mesh_permutation gives
 *     perm[internal] = input element index.
 *   - Layouts (row-major, contiguous, device memory, 8-byte aligned):
 *       pressure      [E][G][N]      (time node, then spatial node)
 *       main velocity [3][E][G][N]   (component-major)
 *       dual velocity [3][F][G][N]   (faces in stdg_mesh_faces order, Taylor
 *                                     coefficients of eq. bf_2 about the volume
 *                                     centroid of the dual element, scaled by
 *                                     half its diameter)
 *     N = (p+1)(p+2)(p+3)/6 spatial nodes (j1,j2,j3)/p, j1 fastest then j2,
 *     then j3, on the element's own vertex order (local vertex 0 = reference
 *     origin); G = p_gamma+1 Gauss-Legendre time nodes of [0,1], ascending.
 *   - Streams: a NULL stream is the default stream.  Functions that say
 *     "asynchronous" only enqueue work; the caller keeps the buffers alive
 *     until the stream reaches that point.  The mesh handle owns its device
 *     tables and workspaces and must not be used from two streams at once.
 *   - Ownership: the caller owns every vector it passes; the library never
 *     frees caller memory.
 */
#ifndef STDG_H
#define STDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STDG_OK 0
#define STDG_NOT_CONVERGED 1   /* x holds the last iterate, report filled   */
#define STDG_ERR_ARG -1        /* null pointer, bad size, degree or option  */
#define STDG_ERR_MESH -2       /* degenerate element, non-manifold face,    */
                               /* unmatched periodic face                   */
#define STDG_ERR_NUMERIC -3    /* NaN/Inf or Krylov breakdown               */
#define STDG_ERR_DEVICE -4     /* HIP runtime error                         */
#define STDG_ERR_NOMEM -5      /* host or device allocation failed          */

/* precision of an operator application or of the inner solve */
#define STDG_FP64 0
#define STDG_FP32 1

/* Krylov method */
#define STDG_AUTO 0            /* CG when p_gamma = 0, GMRES otherwise */
#define STDG_CG 1
#define STDG_GMRES 2
#define STDG_CG_TIME 3         /* any p_gamma: S = dt^2 (S^sp (x) I)(I (x) C), so the  */
                               /* space-time system is G independent symmetric      */
                               /* spatial systems (S^sp (x) I) w = b, x = (I (x) C^-1) w */
                               /* solved by CG: same anchored solution, no GMRES    */
#define STDG_BICGSTAB 4        /* BiCGStab (van der Vorst): short recurrences, two */
                               /* operator applies per iteration, no orthogonal     */
                               /* basis; the viscous solve preconditions it with    */
                               /* the space-time diagonal blocks as GMRES does      */

typedef struct stdg_mesh stdg_mesh;

/* Discretisation parameters (Sec. 2.3: degrees; Sec. 2.2: time step). */
typedef struct {
    int32_t p;             /* spatial degree, 1..6                             */
    int32_t p_gamma;       /* time degree, 0..6                                */
    double nu;             /* kinematic viscosity (Picard step only)           */
    double dt;             /* time step Delta t > 0                            */
    int32_t periodic;      /* 1: faces on opposite sides of the box are paired */
                           /* 0: boundary faces carry Dirichlet velocity       */
    double box_lo[3];      /* box used for periodic pairing                    */
    double box_hi[3];
    int64_t anchor_tet;    /* element (input numbering) whose node anchor_node */
    int32_t anchor_node;   /* holds zero pressure at every time node           */
    int32_t reorder;       /* 1: Hilbert-curve renumbering, 0: keep input order */
} stdg_config;

typedef struct {
    int64_t n_tet;              /* E                                          */
    int64_t n_face;             /* all faces (interior first, then boundary)  */
    int64_t n_interior_face;
    int32_t N, G, Nst;          /* N spatial functions, G time nodes, N*G     */
    int32_t n_classes;          /* distinct operator block sets stored        */
    int64_t anchor_internal;    /* internal index of the anchor element       */
    int32_t inner_layout;       /* STDG_LAYOUT_ELEMENT or STDG_LAYOUT_RUN:    */
                                /* layout of the FP32 inner-solve vectors     */
    int64_t inner_len;          /* floats in one such vector                  */
    int32_t inner_per_element;  /* 1: the FP32 PCG iteration streams a table  */
                                /* of 6 N x N FP32 blocks per element (meshes */
                                /* whose elements mostly have their own       */
                                /* blocks: unstructured or curved)            */
} stdg_mesh_info;

/* Layouts of FP32 vectors of the inner (refinement) solve.
 * STDG_LAYOUT_ELEMENT: [E][G][N] like every FP64 vector.
 * STDG_LAYOUT_RUN (p = 1, 2, 3 on meshes whose consecutive 64-element runs
 * each hold one geometry class, e.g. the class-chunked Kuhn cubes; p = 4 on
 * meshes whose runs hold at most 1.5 classes on average): value k of element
 * e = 64 R + l at time node a is entry (((R G + a) (N / w) + k / w) 64 + l) w
 * + k % w with w = 4 if 4 divides N, else 2 if 2 does, else 1; the length is
 * ceil(E / 64) 64 G N and the entries of the missing elements of a ragged
 * last run are zero. */
#define STDG_LAYOUT_ELEMENT 0
#define STDG_LAYOUT_RUN 1

/* Build the primary mesh, its face-based dual mesh (Sec. 2.2.1) and every
 * precomputed operator block (the paper precomputes and stores all coefficient
 * matrices, Sec. 2.8 and Sec. 4).  Inputs are HOST arrays: xyz[n_vert][3]
 * vertex coordinates, tets[n_tet][4] vertex indices (local order is kept).
 * Synchronous.  On success *out owns all device tables.
 * Errors: STDG_ERR_ARG (null/size/degree), STDG_ERR_MESH (inverted or flat
 * element, non-manifold or unmatched periodic face), STDG_ERR_DEVICE/NOMEM. */
int stdg_mesh_build(const double* xyz, int64_t n_vert, const int64_t* tets,
                    int64_t n_tet, const stdg_config* cfg, stdg_mesh** out);

/* Same tables as stdg_mesh_build, kept on the host only: no device memory
 * or HIP call is touched.  Such a handle serves stdg_mesh_info_get,
 * stdg_mesh_permutation, stdg_mesh_faces and stdg_mesh_blocks (inspection of
 * the precomputed operator); the device entry points reject it with
 * STDG_ERR_ARG. */
int stdg_mesh_build_host(const double* xyz, int64_t n_vert, const int64_t* tets,
                         int64_t n_tet, const stdg_config* cfg, stdg_mesh** out);

/* Mesh with curved (isoparametric) elements, Sec. 2.8.  As stdg_mesh_build
 * (host_only != 0: as stdg_mesh_build_host), plus nodes[n_tet][N][3] (HOST):
 * the physical positions of each element's N spatial nodes, in the layout
 * order of the pressure coefficients (reference points (j1, j2, j3)/p, j1
 * fastest, in the element's local vertex frame).  Element i is the image of
 * the reference tetrahedron under x_i(xi) = sum_k nodes[i][k] phi_k(xi);
 * the sub-tetrahedra of its dual elements are the images of the reference
 * sub-tetrahedra (reference face and barycentre), and a face is met by its
 * two elements at equal barycentric coordinates of its vertices, so the
 * nodes on a shared face must coincide (translated on periodic faces).
 * Every integral is exact (reference coordinates, polynomial integrands of
 * degree <= 2p^2 + 3p - 3), so the precompute costs O(p^8) per curved element;
 * elements whose nodes are the affine image of the reference nodes, and
 * whose neighbours' are too, keep the straight precompute and share blocks.
 * Only the pressure system is built on a curved mesh: stdg_pressure_apply,
 * stdg_pressure_solve and the model calls accept it; stdg_picard_step,
 * stdg_dual_from_main, stdg_main_from_dual and stdg_divergence return
 * STDG_ERR_ARG.  When no element is curved the mesh is the straight one.
 * Errors: those of stdg_mesh_build; STDG_ERR_ARG for nodes == NULL;
 * STDG_ERR_MESH when vertex nodes differ from xyz (relative 1e-12), two
 * elements do not share a curved face (relative 1e-9), or an element's map
 * folds (det J at a quadrature point of opposite sign to, or below 1e-12
 * times, its value at the element's barycentre). */
int stdg_mesh_build_curved(const double* xyz, int64_t n_vert, const int64_t* tets,
                           int64_t n_tet, const double* nodes, int32_t host_only,
                           const stdg_config* cfg, stdg_mesh** out);

/* Copy the precomputed pressure-operator tables to host arrays:
 * blocks[n_classes][5][N][N] (dt^2-scaled spatial blocks; block 0 multiplies
 * the element itself, block 1+f the neighbour across local face f),
 * cls[n_tet] class of each element, nbr[n_tet][4] internal neighbour across
 * local face f (-1 on a boundary face), C[G][G] time factor, so that
 * y_i = sum_k B[cls_i][k] X_k C^T with X_k the N x G coefficients of k.
 * Any output pointer may be NULL to skip it. */
int stdg_mesh_blocks(const stdg_mesh* mesh, double* blocks, int32_t* cls,
                     int32_t* nbr, double* C);

/* Sizes of a built mesh. */
int stdg_mesh_info_get(const stdg_mesh* mesh, stdg_mesh_info* info);

/* perm_out[n_tet] (host): perm_out[internal] = input element index. */
int stdg_mesh_permutation(const stdg_mesh* mesh, int64_t* perm_out);

/* Face list (host arrays of length n_face, faces in the library's order):
 * left/right internal element indices (right = -1 on a boundary face) and the
 * local face index (face opposite local vertex f) in each. */
int stdg_mesh_faces(const stdg_mesh* mesh, int64_t* left, int32_t* left_face,
                    int64_t* right, int32_t* right_face);

/* Release a mesh and its device memory (NULL is ignored). */
void stdg_mesh_free(stdg_mesh* mesh);

/* y = S x with S = -(sum_j D_ij M_j^-1 Q_.j), the negated matrix of eq. CS_19
 * (interior faces only; Dirichlet boundary faces do not couple pressures).
 * x, y: device [E][G][N] doubles, must not overlap.  precision STDG_FP64
 * uses the FP64 blocks, STDG_FP32 the FP32 copy of the blocks with FP32
 * arithmetic (inputs and outputs stay FP64).  Asynchronous on `stream`. */
int stdg_pressure_apply(const stdg_mesh* mesh, int32_t precision,
                        const double* x, double* y, void* stream);

/* Same operator with FP32 vectors and FP32 blocks (the inner operator of the
 * iterative-refinement solve).  x, y: device [E][G][N] floats. Asynchronous. */
int stdg_pressure_apply_f32(const stdg_mesh* mesh, const float* x, float* y,
                            void* stream);

#define STDG_PRECOND_NONE 0
#define STDG_PRECOND_BLOCK_JACOBI 1

typedef struct {
    int32_t method;        /* STDG_AUTO, STDG_CG, STDG_GMRES or STDG_CG_TIME  */
    int32_t restart;       /* GMRES restart length m (1..200)                  */
    double rtol;           /* stop at ||b_a - S_a x|| <= rtol ||b_a||          */
    int32_t max_iter;      /* total inner Krylov iterations allowed            */
    int32_t precision;     /* STDG_FP64: plain solve; STDG_FP32: FP32 inner    */
                           /* Krylov solve inside FP64 iterative refinement    */
    double inner_rtol;     /* relative tolerance of each inner solve (FP32)    */
    int32_t max_outer;     /* refinement steps allowed (FP32)                  */
    int32_t check_every;   /* host polls convergence every k iterations (>=1)  */
    int32_t precond;       /* STDG_PRECOND_BLOCK_JACOBI (the default) or       */
                           /* STDG_PRECOND_NONE: preconditioner M of the FP32  */
                           /* CG inner solves on B (x) I (method STDG_CG_TIME, */
                           /* or STDG_CG at p_gamma = 0) for p = 1, 2, 3: M is  */
                           /* each element's own diagonal block of B (its      */
                           /* class's, inverted once per class), used when     */
                           /* every such block is SPD; other solves ignore it */
} stdg_solve_opts;

typedef struct {
    int32_t status;        /* same as the return value                         */
    int32_t outer_iters;   /* refinement steps (1 for FP64)                    */
    int32_t inner_iters;   /* Krylov iterations (all refinement steps)         */
    int32_t applies;       /* operator applications                            */
    double rel_residual;   /* ||b_a - S_a x|| / ||b_a|| in FP64 at exit        */
    double seconds;        /* wall time of the call                            */
    double initial_rel_residual;  /* the same for the initial guess            */
    double fused_iter_us;  /* device time per iteration of the one-kernel FP32 */
                           /* CG (HIP events around its back-to-back launches;  */
                           /* 0 when that kernel did not run)                  */
} stdg_solve_report;

/* y = (B (x) I) x in FP32: the spatial Schur operator B = dt^2 S^sp of
 * eq. CS_19 (F3 factorisation S = B (x) C) on every time node, i.e. the
 * operator of the time-decoupled solve (STDG_CG_TIME) and, times the scalar
 * C, of the p_gamma = 0 solve.  x, y: device floats in the mesh's inner
 * layout (stdg_mesh_info.inner_layout, inner_len entries), 16-byte aligned,
 * not overlapping.  Runs an FP32 MFMA kernel: the element-per-lane kernel
 * when the inner layout is STDG_LAYOUT_RUN (p = 1, 2, 3 on meshes whose
 * 64-element runs each hold one geometry class; p = 4 on meshes whose runs
 * mostly do), the tile kernel of the fused CG iteration otherwise (p = 1, 2,
 * 3); STDG_ERR_ARG when neither applies.  Asynchronous. */
int stdg_pressure_apply_spatial_f32(const stdg_mesh* mesh, const float* x, float* y, void* stream);

/* Moves between FP64 vectors ([E][G][N] doubles, device) and FP32 vectors in
 * the mesh's inner layout (inner_len floats, device): y = (float)(scale x),
 * padding entries set to zero; and x = scale y.  These are the conversions
 * the refinement solve applies around its FP32 inner solves (the residual
 * scaled to unit norm, the correction scaled back).  Asynchronous on
 * `stream`.  Errors: STDG_ERR_ARG (null pointer, host-only mesh). */
int stdg_inner_from_f64(const stdg_mesh* mesh, const double* x, double scale, float* y, void* stream);
int stdg_inner_to_f64(const stdg_mesh* mesh, const float* y, double scale, double* x, void* stream);

/* Fill opts with defaults: AUTO, restart 50, rtol 1e-10, max_iter 20000,
 * FP64, inner_rtol 1e-4, max_outer 30, check_every 8. */
void stdg_solve_opts_default(stdg_solve_opts* opts);

/* Solve the anchored pressure system S_a x = b_a (eq. CS_19 / A2_mod with the
 * pressure fixed at the anchor node at every time node: rows and columns of
 * the anchor replaced by the identity, b_a = b with the anchor entries set to
 * zero).  b, x: device [E][G][N] doubles; x holds the initial guess on entry
 * and the solution (with x_anchor = 0) on exit.  The library solves the
 * equivalent consistent singular system S x = b~ and shifts by a constant per
 * time node.  Synchronises `stream` before returning.  Returns STDG_OK,
 * STDG_NOT_CONVERGED (x = last iterate; also when rtol lies below what FP64
 * rounding of the system allows, the solve then stopping near that floor)
 * or an error. */
int stdg_pressure_solve(const stdg_mesh* mesh, const double* b, double* x,
                        const stdg_solve_opts* opts, stdg_solve_report* report,
                        void* stream);

/* The solve of stdg_pressure_solve without any device allocation, for
 * callers that cannot allocate (tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and report; supported only with
 * precision STDG_FP64 and method STDG_CG (p_gamma = 0) or STDG_CG_TIME (any
 * p_gamma; STDG_AUTO resolves to CG at p_gamma = 0), other options give
 * STDG_ERR_ARG.  Every work buffer (four vectors of E*N_st doubles, the
 * reduction partials and the device scalars) lives in one fixed device array
 * of 35.6 MB that each GPU the library runs on holds until the process ends,
 * so E*N_st may be at most 1,048,576 (STDG_ERR_ARG otherwise).  Every call on
 * a GPU shares that GPU's array, which keeps the last call's contents: calls
 * that overlap on one GPU (two host threads, or two streams) race.  It calls
 * no hipMalloc/hipFree; the host waits on `stream` as stdg_pressure_solve
 * does. */
int stdg_pressure_solve_noalloc(const stdg_mesh* mesh, const double* b, double* x,
                                const stdg_solve_opts* opts, stdg_solve_report* report,
                                void* stream);

/* ---------------------------------------------------------------------------
 * Picard pressure-correction time step (Sec. 2.6, steps 0-6).
 *
 * Readings fixed where the paper is silent (its boundary terms are only in
 * commented-out text): a Dirichlet face's dual element is the single
 * sub-tetrahedron, its velocity is the projection of the nodal Dirichlet data
 * of its element (the goback map with one side), it has no momentum equation
 * and no pressure coupling; the viscous stress uses that data for the jump on
 * the face; Lambda uses the element's own pressure gradient on a boundary
 * sub-tetrahedron; the Rusanov ghost state is the boundary dual velocity.
 */
#define STDG_GUESS_ZERO 0       /* p^{n+1,0} = 0 (the paper's choice)        */
#define STDG_GUESS_PREVIOUS 1   /* p^{n+1,0} = previous slab's pressure      */

/* Krylov start of the pressure-correction solves (eq. A2_mod) of Picard
 * iteration k, from the same solve of the two previous steps kept by the
 * caller in `hist`: h0_k, h1_k = that solve's value one and two steps back
 * (for k = 0 the new pressure p^{n+1,1}, whose unknown is its correction to
 * p^{n+1,0}; for k >= 1 the correction itself).                            */
#define STDG_KRYLOV_ZERO 0         /* zero correction                         */
#define STDG_KRYLOV_PREVIOUS 1     /* h0_k                                    */
#define STDG_KRYLOV_EXTRAPOLATE 2  /* 2 h0_k - h1_k                           */
#define STDG_KRYLOV_LEARNED 3      /* k = 0: 2 h0 - h1 + g d with the network */
                                   /* correction d = s_D MLP(features of h0,  */
                                   /* h1, b) (model section below) and g      */
                                   /* minimising the solve's initial residual */
                                   /* ||b - S x0|| (two FP64 operator applies */
                                   /* and two dot products; g = 0 is the      */
                                   /* extrapolation); k >= 1: 2 h0_k - h1_k   */

typedef struct stdg_model stdg_model;

typedef struct {
    int32_t n_picard;           /* Picard iterations; 0 = p_gamma + 1        */
    int32_t pressure_guess;     /* STDG_GUESS_ZERO or STDG_GUESS_PREVIOUS    */
    stdg_solve_opts pressure;   /* pressure-correction solves (eq. A2_mod)   */
    stdg_solve_opts viscous;    /* viscous solves (eq. A1_mod), FP64 only    */
    int32_t krylov_guess;       /* STDG_KRYLOV_*                              */
    stdg_model* model;          /* STDG_KRYLOV_LEARNED: the trained model     */
    double* hist;               /* device [n_pic][2][E][G][N] or NULL (needed */
                                /* by all guesses but ZERO): per Picard       */
                                /* iteration k, (h0_k, h1_k) on entry, this   */
                                /* step's value and h0_k on exit; zeros       */
                                /* before the first step                      */
    double* rec_b;              /* device [E][G][N] or NULL: receives the     */
                                /* right-hand side of the first pressure solve */
    double* rec_x;              /* device [E][G][N] or NULL: receives         */
                                /* p^{n+1,1} (training data for the model)    */
    double theta;               /* implicitness of the pressure in the        */
                                /* momentum equation, p_gamma = 0 only (Sec.  */
                                /* 2.7, eqs. CS_15_theta/CS_16_theta): the    */
                                /* step carries theta p^{n+1} + (1-theta) p^n */
                                /* in [1/2, 1]; 1 (default) is the scheme of  */
                                /* Sec. 2.6, 1/2 Crank-Nicolson.  With theta  */
                                /* < 1, p must hold p^n on entry, and hist,   */
                                /* rec_x and the solves work on the weighted  */
                                /* pressure; out of range or with p_gamma > 0 */
                                /* the step returns STDG_ERR_ARG              */
} stdg_step_opts;

typedef struct {
    int32_t pressure_iters;     /* Krylov iterations, all Picard iterations  */
    int32_t viscous_iters;
    double max_pressure_residual;
    double max_viscous_residual;
    double seconds;             /* whole step                                 */
    double pressure_seconds;    /* inside the pressure-correction solves      */
    double viscous_seconds;     /* inside the viscous solves                  */
    int32_t pressure_applies;   /* pressure-operator applications             */
    int32_t first_pressure_iters;      /* iterations of the first solve       */
    double first_pressure_seconds;     /* its time, guess included            */
    double first_initial_residual;     /* ||b - S x0|| / ||b|| of its guess   */
    double pressure_fused_iter_us;     /* fused_iter_us over the step's solves */
    double guess_weight_network;       /* g of STDG_KRYLOV_LEARNED (else 0)    */
    int32_t status;             /* the step's return code: STDG_OK, or      */
                                /* STDG_NOT_CONVERGED when a pressure or    */
                                /* viscous solve stopped above its rtol     */
} stdg_step_report;

/* Defaults: n_picard 0, zero pressure guess, solve defaults, viscous rtol
 * 1e-12, zero Krylov guess, no model, no recording. */
void stdg_step_opts_default(stdg_step_opts* opts);

/* Advance one slab.  vhat [3][F][G][N]: dual velocity of slab n on entry, of
 * slab n+1 on exit; vbar [3][E][G][N]: averaged (eq. average) velocity of slab
 * n on entry (used by Mbar^- of eq. A1_mod), of slab n+1 on exit; p [E][G][N]:
 * pressure of slab n on entry (read only with STDG_GUESS_PREVIOUS), of slab
 * n+1 on exit; g_nodal [3][E][G][N]: Dirichlet velocity at the element nodes
 * of slab n+1 (only elements with boundary faces are read; NULL allowed on a
 * mesh without boundary faces).  Device pointers; workspace is owned by the
 * mesh handle.  Meshes with p_gamma > 4 are rejected (STDG_ERR_ARG).
 * Synchronises `stream`.  Returns STDG_OK; STDG_NOT_CONVERGED
 * when the step ran to its end but a pressure or viscous solve stopped above
 * its rtol (the report's residuals say which); or an error. */
int stdg_picard_step(const stdg_mesh* mesh, double* vhat, double* vbar, double* p,
                     const double* g_nodal, const stdg_step_opts* opts,
                     stdg_step_report* report, void* stream);

/* Dual velocity from a main-grid velocity by eq. goback (one-sided on
 * boundary faces): the initial slab's vhat from nodal initial data.
 * vbar [3][E][G][N] -> vhat [3][F][G][N].  Asynchronous. */
int stdg_dual_from_main(const stdg_mesh* mesh, const double* vbar, double* vhat,
                        void* stream);

/* Main-grid velocity from the dual velocity by eq. average.
 * vhat [3][F][G][N] -> vbar [3][E][G][N].  Asynchronous. */
int stdg_main_from_dual(const stdg_mesh* mesh, const double* vhat, double* vbar,
                        void* stream);

/* Discrete divergence sum_{j in S_i} D_ij vhat_j (eq. CS_15), [E][G][N].
 * Asynchronous. */
int stdg_divergence(const stdg_mesh* mesh, const double* vhat, double* div,
                    void* stream);

/* ---------------------------------------------------------------------------
 * Learned Krylov initial guess.
 *
 * The first pressure-correction solve of a step (Sec. 2.6, step 5, after the
 * zero pressure guess of step 0) yields p^{n+1,1}; plain Krylov starts it
 * from zero or from the previous step's value.  With P = p^{n,1} and
 * Pm = p^{n-1,1} (the same quantity one and two steps back) and b the
 * solve's right-hand side, the model corrects the linear extrapolation,
 * element by element:
 *     x0 = 2 P - Pm + s_D * MLP(f_i),
 * f_i (11 N_st + 4 values) = P of element i and of its neighbours across
 * local faces 0..3 (face f opposite local vertex f) divided by s_P; P - Pm
 * of the same five elements divided by s_D; b_i divided by s_B; four
 * neighbour-present flags (missing neighbours give zeros).  s_P, s_D, s_B are
 * the RMS values of P, P - Pm, b over the mesh (1 if zero).  The MLP
 * is affine - SiLU - affine - SiLU - affine with `hidden` units; parameters
 * flat in the order W1 [n_in][hidden], b1, W2 [hidden][hidden], b2,
 * W3 [hidden][n_out], b3 (n_out = N_st).  Training minimises the mean squared
 * error against (x* - 2P + Pm) / s_D with Adam, x* = p^{n+1,1}.  The Krylov solve that follows is
 * unchanged and judges the guess: a poor guess costs iterations, never
 * accuracy.  A model belongs to one mesh shape (E, N_st); its calls run on
 * the given stream and must not overlap on one model.
 */
typedef struct {
    int32_t hidden;            /* units per hidden layer (default 128)        */
    int32_t precision;         /* STDG_FP32 (default) or STDG_FP64            */
    int32_t batch;             /* rows per training mini-batch and per        */
                               /* inference chunk (default 16384)             */
    uint64_t seed;             /* initial weights and sample order            */
    double lr, beta1, beta2, eps;   /* Adam (1e-3, 0.9, 0.999, 1e-8)          */
    double init_scale_out;     /* output-layer initial scale (default 0: the  */
                               /* untrained model is the extrapolation)      */
    int32_t loss;              /* STDG_LOSS_RESIDUAL (default) or STDG_LOSS_MSE */
} stdg_model_config;

/* Training objectives.  MSE: mean squared error of the network output against
 * (x* - 2P + Pm) / s_D over mini-batches of elements.  RESIDUAL: the initial
 * residual of the solve the guess is for, |S (x0 - x*)|^2 / |S (x_e - x*)|^2
 * with x_e = 2P - Pm and x0 = x_e + s_D MLP, one recorded step per Adam step
 * (its gradient goes through S^T; needs batch >= number of elements). */
#define STDG_LOSS_MSE 0
#define STDG_LOSS_RESIDUAL 1

typedef struct {
    int32_t epochs;
    int64_t samples;           /* elements x steps per epoch                 */
    double first_loss;         /* mean loss over the first epoch             */
    double last_loss;          /* mean loss over the last epoch              */
    double seconds;
} stdg_train_report;

void stdg_model_config_default(stdg_model_config* cfg);

/* Allocate a model for meshes shaped like `mesh` (device memory: parameters,
 * Adam moments and batch activations, about 4 * batch * (n_in + 6 hidden)
 * bytes in FP32).  Weights: seeded uniform Glorot, output layer scaled by
 * init_scale_out, zero biases.  STDG_ERR_ARG for bad sizes, STDG_ERR_NOMEM. */
int stdg_model_create(const stdg_mesh* mesh, const stdg_model_config* cfg, stdg_model** out);
int stdg_model_free(stdg_model* model);
int stdg_model_info(const stdg_model* model, int64_t* n_params, int32_t* n_in, int32_t* n_out);

/* Host copies of the flat parameters / last gradient (doubles); set_params
 * also clears the Adam state.  Synchronous. */
int stdg_model_set_params(stdg_model* model, const double* host);
int stdg_model_get_params(const stdg_model* model, double* host);
int stdg_model_get_grads(const stdg_model* model, double* host);

/* Feature rows F [E][n_in] (device doubles) of P, Pm, B (device [E][G][N]).
 * Asynchronous. */
int stdg_model_features(stdg_model* model, const stdg_mesh* mesh, const double* P, const double* Pm,
                        const double* B, double* F, void* stream);

/* Y [n][n_out] = MLP(F [n][n_in]) for 1 <= n <= batch rows (device doubles;
 * an FP32 model converts).  Asynchronous. */
int stdg_model_forward(stdg_model* model, const double* F, int64_t n, double* Y, void* stream);

/* Mean squared error of MLP(F) against target [n][n_out] and its gradient
 * (kept in the model for stdg_model_adam_step / get_grads).  Writes the loss
 * to *loss (host).  Synchronises the stream. */
int stdg_model_loss_grad(stdg_model* model, const double* F, const double* target, int64_t n,
                         double* loss, void* stream);

/* The residual objective (STDG_LOSS_RESIDUAL) of one recorded step and its
 * gradient (kept in the model): P, Pm, B, X device [E][G][N] as for training
 * (batch >= E).  Writes the loss to *loss.  Synchronises the stream. */
int stdg_model_residual_loss_grad(stdg_model* model, const stdg_mesh* mesh, const double* P,
                                  const double* Pm, const double* B, const double* X, double* loss,
                                  void* stream);

/* One Adam step (with bias correction) from the stored gradient. */
int stdg_model_adam_step(stdg_model* model, void* stream);

/* Train on n_steps recorded solves: P, Pm, B, X device [n_steps][E][G][N]
 * (for step n: p^{n,1}, p^{n-1,1}, the first solve's right-hand side and
 * p^{n+1,1}; `rec_b`/`rec_x` of stdg_step_opts record the last two).  Each epoch visits every (step, element) sample once in a seeded
 * random order, in mini-batches.  Synchronises the stream. */
int stdg_model_train(stdg_model* model, const stdg_mesh* mesh, int32_t n_steps, const double* P,
                     const double* Pm, const double* B, const double* X, int32_t epochs,
                     stdg_train_report* report, void* stream);

/* x0 = 2P - Pm + s_D * MLP(features) for every element (device [E][G][N]).
 * Asynchronous. */
int stdg_model_predict(stdg_model* model, const stdg_mesh* mesh, const double* P, const double* Pm,
                       const double* B, double* x0, void* stream);

/* Message of the last error on this thread ("" if none). */
const char* stdg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STDG_H */
