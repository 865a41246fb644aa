/* libucns -- MI355X (gfx950) explicit residual evaluation of a high-order
 * unstructured finite-volume solver for the compressible Navier-Stokes
 * equations: least-squares CWENOZ reconstruction, Green-Gauss or least-squares gradients,
 * HLLC/Rusanov + viscous face fluxes, per-cell residual and SSP-RK3 update.
 *
 * The method is the one stated in Sec. 2.2 of "Towards Heterogeneous
 * Exascale CFD with a Single Fortran Code Base" (UCNS3D v4): governing
 * equations (eq. ns), finite-volume update (eq. fv_update), least-squares
 * polynomial (eqs. lsq_poly, lsq_system), CWENOZ blend and weights (eqs.
 * cwenoz_poly, cwenoz_weights), viscous interface gradient (eq.
 * viscous_gradient_penalty), semi-discrete system (eq. semi_discrete), and the
 * per-stage sequence of the paper's time-step algorithm (Algorithm 1).
 *
 * Conventions
 *  - Every call returns an int status; UCNS_OK = 0.  Argument, shape and mesh
 *    errors are reported synchronously; a message is kept per thread and read
 *    with ucns_last_error().  No C++ exception crosses this interface.
 *  - The library owns only the host-side mesh handle.  Every device buffer
 *    (mesh arena, state, workspaces, dt, flags) is allocated by the caller and
 *    passed as a device pointer of the current device; device pointers must be
 *    256-byte aligned (UCNS_EINVAL otherwise).  The library never allocates
 *    device memory.
 *  - Compute calls are asynchronous on the caller's HIP stream; launch errors
 *    are returned as UCNS_EHIP, faults surface at the caller's next sync.
 *  - State U is structure-of-arrays [5][n_cell] float64, conserved variables
 *    (rho, rho u, rho v, rho w, rho E).
 *  - precision: UCNS_F64 (all arithmetic in FP64) or UCNS_F32 (operators,
 *    reconstruction, gradients and fluxes in FP32 with FP32 accumulation;
 *    state, residual and RK update stay FP64).
 *  - Face states: each cell's point values at its own face quadrature
 *    points in the precision's type, one row per point slot (lf, q):
 *    [NFMAX][QMAX][n_pad][5], n_pad = n_cell rounded up to a multiple of 64
 *    (ucns_workspace_elems counts the padding);
 *    slot (lf, q) holds the value at point q of local face lf, the points
 *    numbered in the owner's order on both sides of a face (owner = lower
 *    cell id); face fluxes [n_face][5];
 *    gradients [12][n_cell] (row 3*var + dir, var in u, v, w, T).
 *  - A handle may be used by several threads for compute calls at once;
 *    ucns_mesh_upload and ucns_mesh_free must not race with other calls on it.
 */
#ifndef UCNS_H
#define UCNS_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ucns_mesh ucns_mesh;
typedef struct ihipStream_t* ucns_stream; /* a hipStream_t; NULL = default stream */

enum {
    UCNS_OK = 0,
    UCNS_EINVAL = -1,  /* bad argument, size or alignment */
    UCNS_EMESH = -2,   /* invalid mesh: non-positive volume, non-manifold or unmatched face */
    UCNS_ERANK = -3,   /* a central stencil stays rank deficient, or a cell's least-squares gradient fit is singular */
    UCNS_EHIP = -4,    /* HIP runtime error */
    UCNS_ENOMEM = -5,  /* caller buffer too small */
    UCNS_ESTATE = -6,  /* call out of order (e.g. compute before upload) */
    UCNS_ENUM = -7     /* NaN/Inf or non-positive dt detected */
};

enum { UCNS_TET = 4, UCNS_PYR = 5, UCNS_PRISM = 6, UCNS_HEX = 8 };
enum { UCNS_F64 = 0, UCNS_F32 = 1 };
enum { UCNS_RUSANOV = 0, UCNS_HLLC = 1 };
enum { UCNS_GRAD_GREEN_GAUSS = 0, UCNS_GRAD_LSQ = 1 };
enum { UCNS_BC_NONE = 0, UCNS_BC_DIRICHLET = 1, UCNS_BC_TRANSMISSIVE = 2, UCNS_BC_WALL = 3, UCNS_BC_SYMMETRY = 4 };

/* Mesh description (host arrays, read during ucns_mesh_build only).
 * Cell vertex order: VTK for tet and hex; prism: bottom triangle (0,1,2)
 * counter-clockwise seen from the top, then (3,4,5) above it; pyramid: base
 * (0..3) as a hex bottom, apex 4.  Periodic axes (period > 0) list one copy
 * of each periodic vertex; a cell's coordinates are the images nearest its
 * first vertex.  Boundary faces list their vertices in any order; tags 1..7. */
typedef struct {
    int64_t n_vert;
    const double* xyz;        /* [n_vert][3] */
    int64_t n_cell;
    const uint8_t* type;      /* [n_cell] UCNS_TET .. UCNS_HEX */
    const int64_t* cell_ptr;  /* [n_cell+1] */
    const int64_t* cell_vtx;
    double period[3];
    int64_t n_bface;
    const int64_t* bface_ptr; /* [n_bface+1] */
    const int64_t* bface_vtx;
    const int32_t* bface_tag;
} ucns_mesh_desc;

/* Reconstruction options.  order r = 2, 3 or 4 (P2, P3, P4 = CWENOZ5);
 * central stencil round(stencil_factor K(r,3)) cells (closed over distance
 * ties); one directional stencil per face, linear with 8 cells at P2/P3,
 * quadratic with 20 cells at P4 (closed over ties; Sec. 2.2); triangle faces
 * use the 3-point rule, quadrilateral faces r x r Gauss points.  P4 is built
 * for meshes of quadrilateral faces only (UCNS_EINVAL otherwise). */
typedef struct {
    int order;              /* 2, 3 or 4 */
    double lambda_c;        /* central linear weight before normalisation, 1000 */
    double eps;             /* epsilon of the nonlinear weights, 1e-12 */
    int max_layers;         /* vertex-neighbour layers searched, 3 */
    double stencil_factor;  /* central stencil size over K(r,3), 2 (<= 0 also means 2) */
} ucns_recon_opts;

/* Physics: nondimensional with rho_ref = u_ref = L = 1, p_ref = 1/(gamma M^2),
 * T = gamma M^2 p / rho, mu = 1/Re, kappa = mu / ((gamma-1) M^2 Pr). */
typedef struct {
    double gamma, mach, reynolds, prandtl;
    int viscous;        /* 0 Euler, 1 Navier-Stokes */
    int flux;           /* UCNS_RUSANOV or UCNS_HLLC */
    int grad;           /* viscous cell gradients: UCNS_GRAD_GREEN_GAUSS (0) or UCNS_GRAD_LSQ */
} ucns_phys;

/* Boundary condition per face tag 1..7 (index 0 unused); the paper lists the
 * conditions (Sec. 3.6, boundary conditions) but not their form.  The ghost
 * state across a boundary face, at each Gauss point:
 *  - UCNS_BC_DIRICHLET: state[tag] (inflow, far field);
 *  - UCNS_BC_TRANSMISSIVE (also any other kind): the owner's cell average;
 *  - UCNS_BC_WALL (no-slip, adiabatic): the interior point state with its
 *    velocity reversed;
 *  - UCNS_BC_SYMMETRY: the interior point state with its momentum reflected
 *    in the face plane, m - 2 (m . n) n; the viscous face gradient is the
 *    mean of the cell's gradient and its mirror image (no shear stress, no
 *    heat flux through the plane).  Other kinds use the cell's own gradient.
 * Cell gradients use the same ghosts with the cell average as the interior
 * state. */
typedef struct {
    int kind[8];
    double state[8][5]; /* conserved state for UCNS_BC_DIRICHLET */
} ucns_bc;

/* Troubled-cell gate for ucns_reconstruct.  A cell taken as smooth uses the
 * linear central polynomial and skips the directional stencils, smoothness
 * indicators and nonlinear weights; the others take full CWENOZ.  Either a
 * precomputed mask (1 = smooth) or the network's parameters (the network then
 * runs inside the reconstruction kernel on each cell's features, smooth when
 * sigmoid(z) < theta); not both.  mask_out (may be NULL) records the
 * network's decisions.  A NULL gate = full CWENOZ everywhere.  Labels are
 * not produced with a gate. */
typedef struct {
    const uint8_t* mask;    /* device [n_cell] or NULL */
    const void* mlp_image;  /* device image written by ucns_mlp_pack, or NULL */
    uint8_t* mask_out;      /* device [n_cell] or NULL */
} ucns_gate;

/* Gate network parameter block (float32) offsets: mu[16] isig[16]
 * W1[16][64] b1[64] W2[64][64] b2[64] w3[64] b3 theta; inputs are the 12
 * features standardised as (f - mu) * isig, W1[k][n] maps input k to hidden
 * unit n, W2[i][n] hidden i to hidden n. */
enum {
    UCNS_MLP_MU = 0, UCNS_MLP_ISIG = 16, UCNS_MLP_W1 = 32, UCNS_MLP_B1 = 1056, UCNS_MLP_W2 = 1120,
    UCNS_MLP_B2 = 5216, UCNS_MLP_W3 = 5280, UCNS_MLP_B3 = 5344, UCNS_MLP_THETA = 5345, UCNS_MLP_NPARAM = 5348,
    UCNS_MLP_IMAGE_BYTES = 13312
};

const char* ucns_last_error(void);

/* ---------------------------------------------------------------- mesh */

/* Builds, on the host in FP64 and with n_threads threads (0 = hardware), the
 * faces (periodic matching, owner = lower cell id), cell and face geometry,
 * face quadrature, the zero-mean scaled monomial basis, the central and
 * directional stencils and their least-squares operators B = A^+ diag(|V_m|)
 * (eq. lsq_system solved by QR), the smoothness-indicator matrices and the
 * basis values at each cell's face quadrature points.  Errors: UCNS_EINVAL,
 * UCNS_EMESH, UCNS_ERANK.  *out is owned by the caller; free with
 * ucns_mesh_free. */
int ucns_mesh_build(const ucns_mesh_desc* desc, const ucns_recon_opts* opts, int n_threads, ucns_mesh** out);
void ucns_mesh_free(ucns_mesh* mesh);

/* info[0..15]: n_cell, n_face, K (unknowns), QMAX (points per face slot),
 * NFMAX (max faces per cell), padded central stencil, max directional stencils per
 * cell, padded directional stencil, n_boundary_faces, dropped directional
 * stencils, min central stencil size, max central stencil size, order,
 * KD (unknowns of a directional polynomial: 3 linear, 9 quadratic), 0, 0. */
int ucns_mesh_info(const ucns_mesh* mesh, int64_t* info);

/* Bytes of the device arena holding all mesh arrays for one precision (at
 * order 4 also a scratch region of 64 bytes per cell that ucns_reconstruct
 * writes). */
int ucns_mesh_arena_bytes(const ucns_mesh* mesh, int precision, size_t* bytes);

/* Largest byte span that one buffer descriptor of the reconstruction
 * kernels covers for a mesh of n_cell cells with n_unknowns basis terms (9 at
 * P2, 19 at P3) and n_face_slots faces per cell (6 with hexahedra), in the
 * given precision; a host-side query, no device work.  The kernels address
 * each array through descriptors with 32-bit offsets, so ucns_reconstruct and
 * ucns_gate_features return UCNS_EINVAL for a mesh whose span exceeds
 * 0xffffffff bytes (at P2: about 59M cells in FP64, 107M in FP32).  Writes
 * *span; UCNS_EINVAL for a NULL span, a negative n_cell or non-positive
 * counts. */
int ucns_recon_span_bytes(int64_t n_cell, int precision, int n_unknowns, int n_face_slots, uint64_t* span);

/* Copies the packed mesh arrays of one precision into the caller's device
 * arena (256-byte aligned, at least ucns_mesh_arena_bytes) on stream; the
 * handle keeps the pointer.  The arena must outlive every later compute call
 * with that precision. */
int ucns_mesh_upload(ucns_mesh* mesh, int precision, void* arena, size_t bytes, ucns_stream stream);

/* The handle forgets the device arena of one precision (no device work), so
 * that the caller may free it; calls that need that precision then return
 * UCNS_ESTATE until the next upload.  The precision-independent calls
 * (ucns_dt, ucns_diag_ke) read the FP64 arena while one is uploaded, else the
 * FP32 one: release an arena before freeing it. */
int ucns_mesh_release(ucns_mesh* mesh, int precision);

/* Host-side inspection (for verification): cell-to-face table
 * c2f[c*6+lf] = 2*face + side (-1 unused); face cells [n_face][2] (-1 - tag
 * on a boundary side); face quadrature points [n_face][QMAX][3] in the
 * owner's frame; face shift [n_face][3] (neighbour frame = owner frame -
 * shift); stencils and FP64 operators of one cell: central ids (up to 128),
 * directional ids dir[s*32 + j] (up to 32 per stencil), Bc[K][ncen],
 * Bd[(s*KD + k)*32 + j], O[K][K], Phi[NFMAX][QMAX][K]. */
int ucns_mesh_faces(const ucns_mesh* mesh, int32_t* c2f, int64_t* fcell, double* qp, double* shift);
int ucns_mesh_cell_geometry(const ucns_mesh* mesh, double* vol, double* cen, double* hbasis);
int ucns_mesh_stencil(const ucns_mesh* mesh, int64_t cell, int64_t* central, int32_t* ncen, int64_t* dir,
                      int32_t* ndir, int32_t* dface);
int ucns_mesh_operators(const ucns_mesh* mesh, int64_t cell, double* Bc, double* Bd, double* O, double* Phi);
/* Least-squares gradient weights of one cell, G[6][3] by local face slot
 * (host memory, caller-owned; zero for absent slots): grad W_c =
 * sum_lf G[lf] (W_lf - W_c), W_lf the face neighbour's value or the boundary
 * ghost's.  UCNS_EINVAL for a NULL mesh or G or a cell out of range. */
int ucns_mesh_gradient_weights(const ucns_mesh* mesh, int64_t cell, double* G);

/* --------------------------------------------------------- workspaces */

/* Element counts of the caller-owned workspaces: face_state, face_flux,
 * gradW (in the precision's type) and the reduction scratch (float64). */
int ucns_workspace_elems(const ucns_mesh* mesh, int64_t* face_state, int64_t* face_flux, int64_t* gradW,
                         int64_t* reduce_scratch);

/* ------------------------------------------------------------- compute */

/* Time step (reading of the paper's compute_time_step, Listing 1):
 * dt = cfl * min_i h_i / (|u_i| + c_i), h_i = 6|V_i| / sum_f |S_f|; with
 * viscosity also dt <= cfl * min_i rho_i h_i^2 / (2 mu max(4/3, gamma/Pr)).
 * Deterministic two-pass minimum; writes *dt_dev (device scalar). */
int ucns_dt(const ucns_mesh* mesh, const ucns_phys* phys, const double* U, double cfl, double* reduce_scratch,
            double* dt_dev, ucns_stream stream);

/* Reconstruction (Sec. 2.2, eqs. lsq_system, cwenoz_poly, cwenoz_weights):
 * per cell and conserved variable, central and directional least-squares
 * coefficients from stencil jumps, smoothness indicators, WENO-Z nonlinear
 * weights, blend, and the polynomial values at the cell's face quadrature
 * points written to face_state.  Positivity of density and pressure at every
 * point is enforced with the fallback gated-linear -> full CWENOZ -> first
 * order, run as a second pass over the cells that need it; flags[c]
 * (device [n_cell], required) records bit0 linear taken, bit1 CWENOZ
 * fallback, bit2 first-order fallback.  label (device float [n_cell],
 * may be NULL; only without a gate) receives max over variables and stencils
 * of |omega - lambda|.  At order 4 the call first copies U, cell-interleaved,
 * into a scratch region of the mesh's arena (64 bytes per cell, part of
 * ucns_mesh_arena_bytes): two order-4 calls with one mesh and precision
 * must not overlap (e.g. on two streams). */
int ucns_reconstruct(const ucns_mesh* mesh, const ucns_phys* phys, const double* U, int precision,
                     const ucns_gate* gate, void* face_state, uint8_t* flags, float* label, ucns_stream stream);

/* Cell gradients of W = (u, v, w, T) from cell averages, gradW [12][n_cell]
 * (row 3*var + dir), by the method phys->grad names:
 *  - UCNS_GRAD_GREEN_GAUSS: face value the mean of the two cells, ghost state
 *    on boundaries;
 *  - UCNS_GRAD_LSQ: the least-squares gradients the paper's viscous terms use
 *    (Sec. 2.2), read as the linear fit over the face neighbours
 *    with weights 1/|d|^2 (d the centroid offset, across periodic seams); a
 *    boundary face enters as its ghost state at the centroid's mirror image
 *    in the face plane, which carries the boundary condition into the fit
 *    (no-slip: zero wall velocity; adiabatic wall and transmissive outflow:
 *    zero normal derivative).  The fit's weights per face slot are built
 *    with the mesh (UCNS_ERANK there if a cell's fit is singular).
 * Any other phys->grad returns UCNS_EINVAL. */
int ucns_gradients(const ucns_mesh* mesh, const ucns_phys* phys, const ucns_bc* bc, const double* U,
                   int precision, void* gradW, ucns_stream stream);

/* The reconstruction of ucns_reconstruct and the gradients of
 * ucns_gradients (by phys->grad, Green-Gauss or least squares) of the same U
 * in one pass: each cell forms its gradient after its face-point values,
 * from the face neighbours its central stencil has just read (Sec. 2.2: the
 * viscous terms' cell gradients).  The arguments are those of the two calls,
 * except that the boundary table bc_device is a ucns_bc in DEVICE memory
 * (read by the boundary cells' lanes; NULL: every boundary transmissive) and
 * that there is no label output.  Order 2 only: UCNS_EINVAL for order 3 or 4
 * (use the two calls) or an unknown phys->grad.  The gradients differ from
 * ucns_gradients' by rounding only (the Green-Gauss weight n |S| / (2 |V|)
 * of each face slot is stored with the mesh, and a symmetry plane's normal
 * is taken from it). */
int ucns_reconstruct_gradients(const ucns_mesh* mesh, const ucns_phys* phys, const ucns_bc* bc_device,
                               const double* U, int precision, const ucns_gate* gate, void* face_state,
                               uint8_t* flags, void* gradW, ucns_stream stream);

/* Face fluxes (Sec. 2.2, eq. fv_update and eq. viscous_gradient_penalty with
 * alpha = 4/3): F_f = |S_f| sum_q w_q (F_c(U_L, U_R; n) - F_v), HLLC or
 * Rusanov convective flux; one lane per face sums its Gauss points.
 * U (device double [5][n_cell]) supplies the ghost state of transmissive
 * boundary faces (the owner's cell average).  gradW may be NULL for Euler.
 * face_flux [n_face][5]. */
int ucns_face_flux(const ucns_mesh* mesh, const ucns_phys* phys, const ucns_bc* bc, const double* U,
                   const void* face_state, const void* gradW, int precision, void* face_flux, ucns_stream stream);

/* Residual R_i = -(1/|V_i|) sum_f s_if F_f (eq. fv_update), a per-cell gather
 * over the cell's faces in fixed local order (no atomics).  R [5][n_cell]. */
int ucns_residual(const ucns_mesh* mesh, const void* face_flux, int precision, double* R, ucns_stream stream);

/* SSP-RK3 stage s (Shu-Osher): U <- a_s U0 + b_s (U + dt R) with
 * (a, b) = (0, 1), (3/4, 1/4), (1/3, 2/3); dt read from the device scalar.
 * Stage 0 also stores the incoming U (the step's U^n) into U0, which stages 1
 * and 2 then read. */
int ucns_rk_stage(const ucns_mesh* mesh, int stage, const double* dt_dev, double* U0, const double* R,
                  double* U, ucns_stream stream);

/* ucns_residual followed by ucns_rk_stage in one pass (R is not stored);
 * same U0 convention as ucns_rk_stage. */
int ucns_residual_rk_stage(const ucns_mesh* mesh, const void* face_flux, int precision, int stage,
                           const double* dt_dev, double* U0, double* U, ucns_stream stream);

/* The residual fused with stage s (0 .. 4) of the five-stage fourth-order
 * SSP Runge-Kutta method of Spiteri and Ruuth (the integrator family of
 * Sec. 2.2), Shu-Osher form, R = R(U) of the current U:
 *   u1 = u0 + b10 dt R(u0);  u2 = a20 u0 + a21 u1 + b21 dt R(u1);
 *   u3 = a30 u0 + a32 u2 + b32 dt R(u2);  u4 = a40 u0 + a43 u3 + b43 dt R(u3);
 *   u5 = a52 u2 + a53 u3 + b53 dt R(u3) + a54 u4 + b54 dt R(u4)
 * with the published coefficients.  W (device double [4][5][n_cell],
 * caller-owned) keeps u0, u2, u3 and R(u3) between the stages of a step;
 * dt is read from the device scalar. */
int ucns_residual_ssp54_stage(const ucns_mesh* mesh, const void* face_flux, int precision, int stage,
                              const double* dt_dev, double* W, double* U, ucns_stream stream);

/* The last SSP-RK3 stage (ucns_residual_rk_stage with stage 2) fused with the
 * two reductions a step ends with, taken on the new U while it is in
 * registers: the time step of the next step (as ucns_dt with cfl) into
 * *dt_next_dev and the kinetic energy (as ucns_diag_ke) into *ke_dev, each a
 * deterministic two-pass reduction (per-block partials in reduce_scratch,
 * then one small kernel).  dt_next_dev may equal dt_dev. */
int ucns_residual_rk_final(const ucns_mesh* mesh, const ucns_phys* phys, const void* face_flux, int precision,
                           const double* dt_dev, double* U0, double* U, double cfl, double* reduce_scratch,
                           double* dt_next_dev, double* ke_dev, ucns_stream stream);

/* Health check of a run: waits for the stream, then reads the device time
 * step that ucns_dt or ucns_residual_rk_final wrote.  Those reductions write
 * NaN when any cell's admissible step is NaN or not positive, which happens
 * exactly when a state is NaN/Inf or has non-positive density or pressure;
 * the time step is the run's device status word.  Returns UCNS_ENUM in that
 * case (and for an infinite step), UCNS_EHIP if the stream reports an
 * asynchronous error, UCNS_OK otherwise.  Synchronous (a host round trip):
 * call it every few steps, not every stage. */
int ucns_check(const double* dt_dev, ucns_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * operation as ucns_residual_rk_final, with the same arguments except that
 * there is no reduce_scratch.  Its per-block partials live in a fixed device
 * array inside the library (4 MiB per GPU, held until the process ends), so
 * this call allocates nothing and calls no allocating routine; the caller
 * still passes U, U0, face_flux and the device scalars.  Limit: meshes of at
 * most 67,108,864 cells (262,144 blocks of 256); larger ones return
 * UCNS_EINVAL.  Every call on one GPU shares that GPU's array (nothing in it
 * needs to start at zero: each call writes every partial it reads), so calls
 * that overlap on one GPU, e.g. on two streams, race. */
int ucns_residual_rk_final_noalloc(const ucns_mesh* mesh, const ucns_phys* phys, const void* face_flux,
                                   int precision, const double* dt_dev, double* U0, double* U, double cfl,
                                   double* dt_next_dev, double* ke_dev, ucns_stream stream);

/* Kinetic energy sum |V| |m|^2 / (2 rho) / sum |V| (deterministic two-pass
 * sum in a fixed order); writes *ke_dev. */
int ucns_diag_ke(const ucns_mesh* mesh, const double* U, double* reduce_scratch, double* ke_dev,
                 ucns_stream stream);

/* Solenoidal and dilatational dissipation rates of the Taylor-Green
 * diagnostics (Sec. 4.2; the histories compared in Sec. 5.1), from the cell
 * velocity gradients of a preceding ucns_gradients call in the same
 * precision (gradW [12][n_cell], rows 3*var + dir):
 *   eps_s = (mu/|Omega|) sum |V| |curl u|^2,
 *   eps_d = (4 mu / (3 |Omega|)) sum |V| (div u)^2,   mu = 1/Re,
 * each a deterministic two-pass sum in a fixed order (reduce_scratch as for
 * ucns_diag_ke).  Writes eps_dev[0] = eps_s, eps_dev[1] = eps_d (device
 * doubles).  UCNS_EINVAL without a Reynolds number. */
int ucns_diag_dissipation(const ucns_mesh* mesh, const ucns_phys* phys, const void* gradW, int precision,
                          double* reduce_scratch, double* eps_dev, ucns_stream stream);

/* ---------------------------------------------------------------- gate */

/* The gate is this library's addition to the paper's method: a learned
 * troubled-cell indicator that lets smooth cells skip the work of
 * eq. cwenoz_weights.  Twelve features per cell (row-major [n_cell][12],
 * float32, computed in the precision's arithmetic): for v in (rho, rho E),
 * log(1e-12 + x) of the max and mean of |v_m - v_i|/|v_i| over the central
 * stencil, of h |grad p_opt| / |v_i|, and of the max/mean/min over face
 * neighbours of |v_j - v_i - grad p_opt . (c_j - c_i)| /
 * (|v_j - v_i| + h |grad p_opt| + 1e-12 |v_i|). */
int ucns_gate_features(const ucns_mesh* mesh, const double* U, int precision, float* features, ucns_stream stream);

/* Network 12 -> 64 -> 64 -> 1 (ReLU, sigmoid output) on BF16 matrix cores
 * with FP32 accumulation, on n feature rows: prob = sigmoid(z); ucns_gate_mask
 * writes mask = (prob < theta), 1 = smooth. */
int ucns_mlp_forward(const float* params, const float* features, int64_t n, float* prob, ucns_stream stream);

/* Packs a parameter block into the image the fused gate of ucns_reconstruct
 * reads (UCNS_MLP_IMAGE_BYTES bytes of device memory, 256-byte aligned, owned
 * by the caller): the BF16 weights already in the matrix-core operand layout
 * (so each wave loads its fragments directly, with no per-block conversion)
 * and the FP32 vectors.  Call again whenever the parameters change. */
int ucns_mlp_pack(const float* params, void* image, ucns_stream stream);
int ucns_gate_mask(const float* params, const float* features, int64_t n, uint8_t* mask, ucns_stream stream);

/* One training step on a batch of n rows (labels 0/1 as float): forward,
 * class-weighted binary cross-entropy (weight pos_weight on label 1),
 * backward with BF16 matrix-core products and FP32 accumulation, and Adam
 * (beta 0.9/0.999, eps 1e-8, FP32 master weights in params, step t >= 1).
 * grads receives the batch gradient (parameter layout), adam_state holds m
 * then v (2 x UCNS_MLP_NPARAM floats), loss_dev the mean loss.  Only the
 * slots W1 .. b3 are trained; mu, isig and theta are the caller's.  The
 * batch is split over up to 64 one-wave blocks whose gradient partials are
 * summed in block order, so the result depends on n and the data only.  The
 * partials live in a fixed 1.3 MiB device array per GPU: steps on one GPU
 * must be ordered (one stream); overlapping steps race. */
int ucns_mlp_train_step(float* params, float* grads, float* adam_state, const float* features,
                        const float* labels, int64_t n, float pos_weight, float lr, int t, float* loss_dev,
                        ucns_stream stream);

#ifdef __cplusplus
}
#endif
#endif
