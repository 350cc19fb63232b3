/*
 * hfv.h -- C ABI of the MI355X hybrid finite-volume reconstruction library.
 *
 * The library implements the per-cell reconstruction stage of the hybrid
 * scheme of Tong & Tsoutsanis, "A Hybrid Finite-Volume Reconstruction
 * Framework for Efficient High-Order Shock-Capturing on Unstructured Meshes"
 * (arXiv 2510.25906):
 *   - linear least-squares reconstruction with per-cell pseudo-inverses
 *     (Section 2.1, Eqs. AVGVariables1-dofMatrix),
 *   - the single-step numerical admissibility detector, NAD (Section 2.5,
 *     Eqs. DMP-NADDeactivatedCriteria_2) tagging each cell linear / CWENOZ /
 *     MUSCL, with its von Neumann neighbourhood,
 *   - CWENOZ on weakly non-smooth cells (Section 2.3),
 *   - Barth-Jespersen limited MUSCL on discontinuous cells (Section 2.2),
 *   - the Harten bound check with first-order fallback (Section 2.4,
 *     Eq. harten_jump_fix),
 *   - face Gauss-point states, HLLC / HLL fluxes and the residual
 *     (Section 2, Eq. EulerEquationsDetails with F_v = 0).
 *
 * Conventions shared by every entry point:
 *   - Status codes only; nothing throws or exits across the ABI.
 *   - Host pointers (mesh, stencils, params) are read during the call and
 *     not retained.  Device pointers are caller-owned and must stay valid
 *     until the work enqueued on `stream` has completed.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Hot calls only enqueue work; they never synchronise the host.
 *   - Precision (64 or 32) is fixed at create; every device array of
 *     conserved variables, states and residuals is double or float to match.
 *   - Conserved variables are structure-of-arrays [nvar][n_cells] with
 *     nvar = dim + 2: (rho, rho u, rho v[, rho w], E).
 *   - Face Gauss-point states are cell-major, [ngp_cell_max][nvar][n_cells]
 *     (ngp_cell_max = HFV_Q_NGP_CELL_MAX): slot g of cell c is the g-th
 *     Gauss point on the faces of c, its faces taken in increasing face id
 *     and each face's points in that face's quadrature order (the same order
 *     for both cells of a face).  Slots beyond a cell's own count are left
 *     untouched.  Face f's points start at slot (t & 255) of face_cells[f][0]
 *     and at slot ((t >> 8) & 255) of face_cells[f][1], t = the f-th entry of
 *     table HFV_T_FACE_SLOTS; a boundary face has no right state of its own
 *     (its transmissive ghost is the left state).
 *   - A context is not thread-safe; calls that overlap on one context race.
 */
#ifndef HFV_H
#define HFV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hfv_ctx hfv_ctx;

typedef enum {
  HFV_OK = 0,
  HFV_ERR_PARAM = -1, /* invalid parameter value or NULL argument */
  HFV_ERR_MESH = -2,  /* inconsistent mesh or stencil data */
  HFV_ERR_RANK = -3,  /* a least-squares system is rank deficient / ill conditioned (cell id in last_error) */
  HFV_ERR_DTYPE = -4, /* precision mismatch */
  HFV_ERR_HIP = -5,   /* a HIP runtime call failed */
  HFV_ERR_OOM = -6,   /* device allocation failed */
  HFV_ERR_STATE = -7  /* call not valid in the context's state */
} hfv_status;

/* element types: local vertex orders
 *   TRI (0,1,2) and QUAD (0,1,2,3) counter-clockwise; TET positively oriented;
 *   PYR base (0..3) counter-clockwise seen from the apex 4; PRISM bottom (0,1,2),
 *   top (3,4,5); HEX bottom (0..3), top (4..7).  Faces must be planar. */
enum { HFV_TRI = 0, HFV_QUAD = 1, HFV_TET = 2, HFV_PYR = 3, HFV_PRISM = 4, HFV_HEX = 5 };
/* scheme modes: the hybrid (Section 2.5) or one scheme everywhere */
enum { HFV_HYBRID = 0, HFV_ALL_LINEAR = 1, HFV_ALL_CWENOZ = 2, HFV_ALL_MUSCL = 3 };
enum { HFV_HLLC = 0, HFV_HLL = 1 };
/* CWENOZ weight form: Z form w_s = l_s (1 + (tau/(eps+SI_s))^b) (default) or the
 * printed placement l_s (1 + tau^b/(eps+SI_s)) of Section 2.3 */
enum { HFV_WENOZ_POW = 0, HFV_LITERAL = 1 };
/* MUSCL slope limiter (Section 2.2; the comparison of Section 3.2): Barth-
 * Jespersen (default) or Venkatakrishnan with eps^2 = (kappa h_c)^3 */
enum { HFV_LIM_BJ = 0, HFV_LIM_VENKAT = 1 };
/* variables the CWENOZ reconstruction acts on (Section 2.3: characteristic,
 * primitive or conserved): conserved (default), or characteristic, face by
 * face: the eigenvectors of the Euler flux Jacobian in the face's normal at
 * the Roe average of the cell and the cell across the face project the
 * stencil data (W = L U), CWENOZ weights are taken per characteristic field,
 * and the values at the face's Gauss points are mapped back (U = R W).
 * The VJP entry points support conserved variables only (HFV_ERR_STATE). */
enum { HFV_CONSERVED = 0, HFV_CHARACTERISTIC = 1 };
/* cell classes written to cell_class[] */
enum { HFV_CLASS_LINEAR = 0, HFV_CLASS_CWENOZ = 1, HFV_CLASS_MUSCL = 2, HFV_CLASS_FIRST_ORDER = 3 };

/* Mesh (Section 2: mixed elements, faces with Gauss quadrature).
 * face_vtx lists each face's vertices oriented so that the right-hand-rule
 * normal points out of face_cells[f][0]; face_cells[f][1] = -1 marks a
 * boundary face (transmissive ghost).  face_shift[f] (optional) gives the
 * periodic image of the right cell: its coordinates plus face_shift[f]*period
 * place it next to the left cell. */
typedef struct {
  int32_t dim, n_vertices, n_cells, n_faces;
  const double *vertices;       /* [n_vertices][dim] */
  const int8_t *cell_type;      /* [n_cells] */
  const int32_t *cell_vtx_off;  /* [n_cells+1] */
  const int32_t *cell_vtx;      /* [cell_vtx_off[n_cells]] */
  const int32_t *face_cells;    /* [n_faces][2] */
  const int32_t *face_vtx_off;  /* [n_faces+1] */
  const int32_t *face_vtx;      /* [face_vtx_off[n_faces]] */
  const int8_t *face_shift;     /* [n_faces][dim] or NULL */
  const double *period;         /* [dim] or NULL (required when shifts are given) */
} hfv_mesh;

/* Stencils (Section 2.1 central stencil of M = 2K cells excluding the cell;
 * Section 2.3 directional stencils, one per face, of Md = 2*dim cells
 * contained in the central stencil; Section 2.2 MUSCL neighbours).  Every
 * entry is a cell id plus an optional periodic image shift (multiplies
 * period).  Padding entries are -1. */
typedef struct {
  int32_t M;                    /* central stencil size, must equal 2K */
  int32_t nf_max;               /* row stride of dir / muscl: 4 in 2D, 6 in 3D */
  int32_t Md;                   /* directional stencil size, must equal 2*dim */
  const int32_t *central;       /* [n_cells][M] */
  const int8_t *central_shift;  /* [n_cells][M][dim] or NULL */
  const int32_t *dir;           /* [n_cells][nf_max][Md] */
  const int8_t *dir_shift;      /* [n_cells][nf_max][Md][dim] or NULL */
  const int32_t *n_dir;         /* [n_cells] directional stencils per cell */
  const int32_t *muscl;         /* [n_cells][nf_max] */
  const int8_t *muscl_shift;    /* [n_cells][nf_max][dim] or NULL */
  const int32_t *n_muscl;       /* [n_cells] */
} hfv_stencils;

/* Parameters.  order_r is the polynomial degree r (order r+1, Section 2.1):
 * 1..6 in 2D (Table 1 runs r = 2, 4, 6), 1..4 in 3D; the VJP entry points
 * are built for r <= 4 (HFV_ERR_PARAM above).
 * NAD margins alpha/beta (Eqs. marginm, marginw), deactivation
 * delta U < (kappa h_c)^n_exp (Eq. NADDeactivatedCriteria), CWENOZ lambda_1',
 * eps, b (Section 2.3), Harten theta, eps (Eq. harten_jump_fix); limiter
 * HFV_LIM_* of the MUSCL reconstruction (kappa also sets the Venkatakrishnan
 * eps^2 = (kappa h_c)^3: the paper quotes kappa = 5 for both).
 * viscous = 1 adds the Navier-Stokes viscous fluxes F_v of Eq.
 * EulerEquationsDetails (Section 2, Eqs. Terms1, sutherlandlaw, HeatConduct,
 * Stresses): temperature T = p / rho, viscosity mu = mu0 (T/T0)^(3/2)
 * (T0 + S) / (T + S) with S = sutherland_S, conduction (mu / Pr) gamma /
 * (gamma - 1) grad T with Pr = prandtl; gradients at the face Gauss points
 * from each side's central least-squares polynomial, averaged with the
 * penalty (visc_alpha / L_int) (U_R - U_L) n of Eq. viscous_jump (alpha =
 * 4/3 in the paper; L_int the distance between the cell centres; no jump at
 * boundary faces); the flux is taken at the mean of the two face states.
 * The VJP entry points and hfv_residual_noalloc refuse viscous contexts
 * (HFV_ERR_STATE). */
typedef struct {
  int32_t order_r, scheme_mode, precision, riemann, cweno_form, limiter, cweno_vars, viscous;
  double gamma, alpha_m, beta_m, alpha_w, beta_w, kappa, n_exp, lambda1_prime, eps_w, b_w,
      tvd_theta, tvd_eps;
  double mu0, T0, sutherland_S, prandtl, visc_alpha;
} hfv_params;

/* Build a context: validates the mesh and stencils, uploads them, and
 * computes on the GPU in FP64 the geometry, the exact least-squares
 * matrices, their pseudo-inverses by Householder QR (computed once,
 * Section 2.1), the directional and MUSCL pseudo-inverses and the
 * oscillation-indicator matrices (Section 2.3); FP32 contexts then keep FP32
 * copies.  Synchronises `stream` once at the end (rank report).
 * Returns HFV_ERR_RANK (cell id in hfv_last_error) for a degenerate stencil.
 * On success *out owns all device tables; release with hfv_destroy. */
hfv_status hfv_create(const hfv_mesh *mesh, const hfv_stencils *st, const hfv_params *p, void *stream,
                      hfv_ctx **out);

/* Change run-time parameters (scheme_mode, riemann, cweno_form, margins,
 * deactivation, CWENOZ and Harten constants).  order_r and precision must
 * equal the values given at create (HFV_ERR_PARAM otherwise).  In an FP64
 * context, the first call that turns the viscous fluxes on in a context
 * created without them allocates their gradient buffer (N x ngp_cell_max x
 * dim x nvar doubles; HFV_ERR_OOM, nothing changed, if that fails); a
 * context created with them has it from hfv_create. */
hfv_status hfv_set_params(hfv_ctx *ctx, const hfv_params *p);

/* Reconstruction (Section 2.5 flowchart): linear candidate and NAD on every
 * cell, tagging of the von Neumann neighbourhood, CWENOZ / MUSCL on the
 * tagged cells through per-class work lists, Harten check on every cell.
 *   U            device [nvar][n_cells] cell averages
 *   face_states  device [ngp_cell_max][nvar][n_cells] output (layout above)
 *   cell_class   device [n_cells] uint8 output (HFV_CLASS_*)
 *   near_margin  device [n_cells] output in the context's precision, or
 *                NULL: how close each cell's class decisions came to their
 *                thresholds, the smallest of these relative distances
 *                (a diagnostic; values near 0 mark decisions that rounding
 *                can flip, e.g. between the FP32 and FP64 paths):
 *                - NAD (Eqs. NADMUSCL, NADCWENOZ, marginm, marginw), per
 *                  conserved variable with a non-zero range R = M - m of the
 *                  cell and its face neighbours: min(|d - delta_w|,
 *                  |d - delta_m|) / max(|m|, |M|, R), d the linear
 *                  candidate's largest excursion past [m, M] at the cell's
 *                  face Gauss points (hybrid mode);
 *                - deactivation (Eq. NADDeactivatedCriteria):
 *                  |dU - (kappa h)^n| / max(dU, (kappa h)^n) (hybrid mode);
 *                - Harten (Eq. harten_jump_fix) at every face Gauss point of
 *                  the linear candidate, density and pressure:
 *                  | |q - q_bar| - theta s | / s, s = max(|q_bar|, eps)
 *                  (hybrid and all-linear modes).
 *                +inf in the all-CWENOZ and all-MUSCL modes, which have no
 *                linear pass.  The Harten checks of the CWENOZ and MUSCL
 *                states are not included.
 * Asynchronous on `stream`. */
hfv_status hfv_reconstruct(hfv_ctx *ctx, const void *U, void *face_states, uint8_t *cell_class, void *near_margin,
                           void *stream);

/* Residual R_i = -(1/|V_i|) sum_f sum_alpha F(U_L, U_R) w_alpha |S_f| of
 * Eq. EulerEquationsDetails (F_v = 0) with HLLC or HLL fluxes (Section 2.4).
 *   R            device [nvar][n_cells] output
 *   face_states  device [ngp_cell_max][nvar][n_cells] output, or NULL to use internal storage
 *   cell_class   device [n_cells] output, or NULL to use internal storage
 * Deterministic: no floating-point atomics. */
hfv_status hfv_residual(hfv_ctx *ctx, const void *U, void *R, void *face_states, uint8_t *cell_class,
                        void *stream);

/* The residual of hfv_residual without any device allocation and without
 * the context's workspace: for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The kernels' scratch (own classes, class lists and their
 * lengths, face fluxes: HFV_Q_NOALLOC_BYTES bytes for this context) is carved
 * from one fixed array of HFV_NOALLOC_SCRATCH_BYTES bytes in the library,
 * one per device, held until the process ends; the library takes its device
 * address during hfv_create.
 *   U, R         device [nvar][n_cells]
 *   face_states  device [ngp_cell_max][nvar][n_cells] output (required)
 *   cell_class   device [n_cells] output (required)
 * The CWENOZ pass always refits its central polynomial here (cwenoz_reuse
 * is ignored), so results equal hfv_residual's to rounding, and bit for bit
 * when cwenoz_reuse is 0.  Every call on one device uses that device's one
 * array: calls that overlap on a device (other streams, other contexts,
 * other threads) race and must be serialised by the caller.
 * Errors: HFV_ERR_PARAM for a NULL pointer or a mesh needing more scratch
 * than the maximum (the message gives both sizes). */
#define HFV_NOALLOC_SCRATCH_BYTES (64u << 20)
hfv_status hfv_residual_noalloc(hfv_ctx *ctx, const void *U, void *R, void *face_states, uint8_t *cell_class,
                                void *stream);

/* Residual with given cell classes (the switches of a previous evaluation
 * held fixed): the reconstruction of each cell follows cell_class, with no
 * NAD and no Harten re-check.  The residual a VJP linearises.
 *   cell_class  device [n_cells] classes (HFV_CLASS_*), read only; a value
 *               above HFV_CLASS_FIRST_ORDER is taken as first order */
hfv_status hfv_residual_frozen(hfv_ctx *ctx, const void *U, const uint8_t *cell_class, void *R, void *stream);

/* One stage of an explicit Runge-Kutta method in Shu-Osher form, the form of
 * the strong-stability-preserving methods of Spiteri and Ruuth that the paper
 * integrates in time with (Section 2.4):
 *   out = a U0 + b U1 + c R, evaluated as (a U0 + b U1) + c R,
 * elementwise over device [nvar][n_cells] arrays in the context's precision
 * (R is a residual from hfv_residual, the step size folded into c).  U0, U1
 * or R may be NULL (the term is left out); any input may alias `out`.
 * Errors: HFV_ERR_PARAM for a NULL `out` or a non-finite coefficient. */
hfv_status hfv_rk_stage(hfv_ctx *ctx, double a, const void *U0, double b, const void *U1, double c, const void *R,
                        void *out, void *stream);

/* Largest spectral radius of the cells' upwind updates,
 *   rate = max_i (|u_i| + c_i) sum_{f of i} |S_f| / |V_i|,
 * of the cell averages U (device [nvar][n_cells]), computed in double and
 * written to out (device, one double).  The explicit step at CFL number nu is
 * nu / rate (Sections 2.4 and 3 fix the CFL number, not its definition): at
 * nu = 1 a forward-Euler step of the first-order upwind scheme is at its
 * positivity limit, and the SSP Runge-Kutta method of hfv_rk_stage keeps
 * strong stability up to its SSP coefficient times that.  A cell whose
 * density or pressure is not positive gives +inf.  A fixed-order two-pass
 * reduction (no atomics) through a buffer allocated at create. */
hfv_status hfv_cfl_rate(hfv_ctx *ctx, const void *U, double *out, void *stream);

/* Vector-Jacobian product of the residual with the cell classes frozen (a
 * project addition, not in the paper):  gU = (dR/dU)^T gR, every switch
 * (class, Harten fallback, limiter argmin, Riemann branch) held at the
 * value the forward evaluation of U takes.
 *   cell_class  device [n_cells] classes from hfv_residual on the same U (a
 *               value above HFV_CLASS_FIRST_ORDER is taken as first order)
 *   gR, gU      device [nvar][n_cells]
 * Either MUSCL limiter is differentiated through its limiting Gauss point and
 * the neighbour that sets the bound. */
hfv_status hfv_residual_vjp(hfv_ctx *ctx, const void *U, const uint8_t *cell_class, const void *gR, void *gU,
                            void *stream);

/* The same product when the caller holds the face states of U (project
 * addition): the frozen forward reconstruction that hfv_residual_vjp runs
 * first is skipped and only the class lists are rebuilt from cell_class.
 *   face_states  device [ngp_cell_max][nvar][n_cells], read only: the states
 *                hfv_residual or hfv_reconstruct wrote for this U and these
 *                classes (other states give the product at those states)
 * The result equals hfv_residual_vjp's up to the rounding of the states (the
 * forward pass may take CWENOZ's central fit from the linear pass).
 * Errors: HFV_ERR_PARAM for a NULL pointer; HFV_ERR_STATE as hfv_residual_vjp. */
hfv_status hfv_residual_vjp_states(hfv_ctx *ctx, const void *U, const uint8_t *cell_class, const void *face_states,
                                   const void *gR, void *gU, void *stream);

/* Queries.  HFV_Q_COUNT_* are the lengths of the CWENOZ, MUSCL and
 * first-order work lists as the last compaction built them (hybrid and
 * all-linear reconstructions, the frozen residual and the VJP): cells that
 * the CWENOZ or MUSCL pass then demotes to first order by the Harten check
 * are still counted in their list, and the all-CWENOZ and all-MUSCL modes,
 * which build no lists, leave them at 0.  The final classes are the
 * cell_class output.  Reading a count synchronises the whole device (every
 * stream) first, then copies the counters. */
enum {
  HFV_Q_N_CELLS = 0, HFV_Q_N_FACES = 1, HFV_Q_N_GP = 2, HFV_Q_NVAR = 3, HFV_Q_K = 4, HFV_Q_M = 5,
  HFV_Q_PRECISION = 6, HFV_Q_DIM = 7, HFV_Q_TABLE_BYTES = 8,
  HFV_Q_COUNT_CWENOZ = 9, HFV_Q_COUNT_MUSCL = 10, HFV_Q_COUNT_FIRST = 11, HFV_Q_NGP_CELL_MAX = 12,
  HFV_Q_NOALLOC_BYTES = 13  /* scratch bytes hfv_residual_noalloc needs for this context */
};
hfv_status hfv_query(const hfv_ctx *ctx, int32_t what, int64_t *out);

/* Copy a precomputed table to host memory (for inspection and tests).
 * Layouts (ctx precision unless stated):
 *   HFV_T_PINV   [K][M][n_cells]   pseudo-inverse with |V_m'| folded in
 *   HFV_T_OI     [K(K+1)/2][n_cells] oscillation-indicator matrix, packed upper triangle
 *   HFV_T_PSIBAR [K][n_cells]      basis means
 *   HFV_T_GEOM   [dim+2][n_cells]  double: centroid, volume, h_c
 *   HFV_T_PDIR   [nf_max][dim][Md][n_cells] directional pseudo-inverses
 *   HFV_T_PMUS   [dim][nf_max][n_cells] MUSCL pseudo-inverses
 *   HFV_T_FACE_SLOTS [n_faces] int32: first Gauss-point slot of each face in
 *                its left (bits 0-7) and right (bits 8-15) cell
 *   HFV_T_GP_XI  [ngp_cell_max][dim][n_cells] each cell's Gauss-point slots
 *                in its own frame, xi = (x - x_c) / h_c (x_c, h_c from
 *                HFV_T_GEOM; periodic images unwrapped), slot order as in the
 *                face states; slots past the cell's Gauss points hold 0
 * `bytes` must equal the table size. */
enum { HFV_T_PINV = 0, HFV_T_OI = 1, HFV_T_PSIBAR = 2, HFV_T_GEOM = 3, HFV_T_PDIR = 4, HFV_T_PMUS = 5,
       HFV_T_FACE_SLOTS = 6, HFV_T_GP_XI = 7 };
hfv_status hfv_copy_table(const hfv_ctx *ctx, int32_t which, void *host_dst, int64_t bytes);

/* Launch configuration of the hot path (results agree to rounding for every
 * valid configuration; classes are identical in FP64).
 *   lanes_per_cell  lanes of a wave sharing one cell in the class-list
 *                   kernels (CWENOZ, MUSCL), which split the variables: 1, 2
 *                   or 4 in 2D; 1 or 5 in 3D
 *   block           threads per block: 64, 128, 192 or 256
 *   list_blocks     blocks of the class-list kernels, which stride over their
 *                   list (>= 1), or 0 for one list entry per lane group and a
 *                   grid that covers every cell
 *   linear_split    mapping of the linear + NAD kernel: 0 = lanes split the
 *                   conserved variables, 1 = lanes split the stencil members
 *                   and Gauss points, 2 = lanes split the polynomial's
 *                   unknowns (rows of the pseudo-inverse) and reduce-scatter
 *                   the Gauss-point sums
 *   linear_lanes    lanes per cell of the linear kernel: as lanes_per_cell
 *                   for linear_split 0; 2, 4 or 8 for 1 and 2
 *   cwenoz_reuse    1: in hybrid mode the linear pass keeps every cell's
 *                   central fit and the CWENOZ pass starts from it (the same
 *                   polynomial, Section 2.3): pays off when CWENOZ cells are
 *                   most of the mesh; 0: the CWENOZ pass refits it
 *   fused_residual  1: one kernel per cell evaluates the Riemann fluxes of the
 *                   cell's faces and sums them (each interior face's flux is
 *                   evaluated by both of its cells, with identical operands, so
 *                   conservation stays exact); 0: face fluxes, then a gather
 *   xcd_remap       1: permute block ids so that the blocks the dispatcher
 *                   places on one XCD (every eighth block) cover one
 *                   contiguous range of cells, lists or faces, and neighbour
 *                   gathers share that XCD's L2; 0: plain block order
 *   muscl_lanes     lanes per cell of the MUSCL / first-order pass: 0 (the
 *                   same as lanes_per_cell), 1 or nvar (or 2 in 2D)
 *   merged_lists    1: in hybrid mode with conserved-variable CWENOZ (and in
 *                   the frozen residual and VJP forward), the CWENOZ launch
 *                   also serves the MUSCL and first-order lists, after its
 *                   own, with lanes_per_cell lanes (muscl_lanes unused); their
 *                   cells fill the waves CWENOZ leaves idle.  0: a launch of
 *                   their own
 *   lists_cell_major 1: the class-list kernels read their per-cell tables
 *                   from cell-major copies ([cell][entry], built at create):
 *                   CWENOZ (conserved variables, two or more lanes per cell)
 *                   its OI matrices, directional ids and fits, basis means and
 *                   Gauss-point coordinates; MUSCL its member ids and fits,
 *                   face neighbours, basis means and Gauss-point coordinates.
 *                   A sparse class list then reads each listed cell's entries
 *                   from consecutive cache lines; 0: from the [entry][cell]
 *                   tables, contiguous across the consecutive cells of a
 *                   dense list
 * hfv_set_launch validates every field (HFV_ERR_PARAM, nothing changed, on
 * an invalid one); hfv_get_launch reads the current configuration. */
typedef struct {
  int32_t lanes_per_cell, block, list_blocks, linear_split, linear_lanes, cwenoz_reuse, fused_residual, xcd_remap,
      muscl_lanes, merged_lists, lists_cell_major;
} hfv_launch;
hfv_status hfv_set_launch(hfv_ctx *ctx, const hfv_launch *cfg);
hfv_status hfv_get_launch(const hfv_ctx *ctx, hfv_launch *cfg);

/* Autotuner (a project addition, not in the paper): times hfv_residual on the
 * caller's state U (device [nvar][n_cells]) under the current parameters for
 * candidate launch configurations, searched one coordinate at a time (linear
 * kernel mapping; class-list kernel lanes, block and grid, in hybrid mode
 * jointly with CWENOZ reuse and with the MUSCL and first-order lists merged
 * into the CWENOZ launch; fused or two-kernel residual; XCD block order; in
 * hybrid mode, without merged lists, the MUSCL lanes; the class-list
 * tables' layout; then the four fastest configurations timed again), and keeps the fastest of that second timing
 * (each timing: after one untimed
 * call, three batches of `reps` calls back to back, reps in [1, 1000]; the
 * median batch's time per call).  Synchronous; it
 * allocates and frees one residual-sized buffer.  `best` (may be NULL)
 * receives the chosen configuration, which is also applied; up to
 * `max_records` (configuration, ms per call) pairs go to `records` (may be NULL
 * when max_records is 0) and the number of configurations timed to
 * `*n_records` (may be NULL).  On failure the starting configuration is
 * restored. */
typedef struct {
  hfv_launch cfg;
  double ms;
} hfv_tune_record;
hfv_status hfv_autotune(hfv_ctx *ctx, const void *U, int32_t reps, hfv_launch *best, hfv_tune_record *records,
                        int32_t max_records, int32_t *n_records, void *stream);

/* Kernel timing with HIP events recorded on the launch stream (timing-only
 * events: recording them issues no system-scope memory fence, so the caches
 * are not written back in the middle of a step; they order nothing).
 * hfv_profile_enable arms up to `capacity` timed launches of the kernels
 * selected by `slot_mask` (bit i = HFV_SLOT_i); capacity 0 disables.
 * HFV_SLOT_CWENOZ times the CWENOZ launch, which also serves the MUSCL and
 * first-order lists when merged_lists is 1 (HFV_SLOT_MUSCL then records
 * nothing in hybrid mode).
 * hfv_profile_read synchronises on the recorded events, writes per-slot sums
 * of the launch durations in milliseconds and launch counts (arrays of
 * HFV_NSLOTS), and re-arms the buffer.  HFV_SLOT_MUSCL times the kernel that
 * serves both the MUSCL and the first-order lists; HFV_SLOT_FLUX the fused
 * residual kernel when fused_residual is 1 (HFV_SLOT_GATHER then records
 * nothing); HFV_SLOT_RESERVED records nothing. */
enum {
  HFV_SLOT_LINEAR = 0, HFV_SLOT_CLASSIFY = 1, HFV_SLOT_CWENOZ = 2, HFV_SLOT_MUSCL = 3, HFV_SLOT_RESERVED = 4,
  HFV_SLOT_FLUX = 5, HFV_SLOT_GATHER = 6, HFV_SLOT_VJP = 7, HFV_NSLOTS = 8
};
hfv_status hfv_profile_enable(hfv_ctx *ctx, int32_t capacity, int32_t slot_mask);
hfv_status hfv_profile_read(hfv_ctx *ctx, double *ms_sum, int64_t *launches);

/* Message of the last failure on this context (or of the last failed
 * create when ctx is NULL); never NULL. */
const char *hfv_last_error(const hfv_ctx *ctx);

void hfv_destroy(hfv_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* HFV_H */
