/* FP64 CPU oracle of the explicit residual evaluation of a high-order
 * unstructured finite-volume solver (CWENOZ reconstruction, Green-Gauss
 * gradients, HLLC/Rusanov + viscous face fluxes, per-cell residual, SSP-RK3).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may call it.  It shares no code with the
 * HIP library; the two meet only through the seeded input arrays.
 *
 * Every array is plain host memory owned by the caller unless stated.
 * All functions return 0 on success, a negative code on error
 * (oracle_last_error() holds a message).
 */
#ifndef UCNS_ORACLE_H
#define UCNS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oracle_mesh oracle_mesh;

typedef struct {
    int64_t n_vert;
    const double* xyz;          /* [n_vert][3] */
    int64_t n_cell;
    const uint8_t* type;        /* 4 tet, 5 pyramid, 6 prism, 8 hex */
    const int64_t* cell_ptr;    /* [n_cell+1] */
    const int64_t* cell_vtx;
    double period[3];           /* 0 = not periodic */
    int64_t n_bface;
    const int64_t* bface_ptr;   /* [n_bface+1] */
    const int64_t* bface_vtx;
    const int32_t* bface_tag;   /* 1..7 */
} oracle_mesh_in;

typedef struct {
    int order;          /* polynomial degree r of the central reconstruction (1 .. 4; 4 on hexahedra only) */
    int tri_qp;         /* quadrature points on triangular faces (3) */
    double lambda_c;    /* central linear weight before normalisation (1000) */
    double eps;         /* epsilon of the nonlinear weights (1e-12) */
    int max_layers;     /* vertex-neighbour layers searched for stencils (3) */
    double stencil_factor; /* central stencil size Mc = round(stencil_factor K(r,3)) (2) */
} oracle_opts;

typedef struct {
    double gamma, mach, reynolds, prandtl;
    int viscous;        /* 0 Euler, 1 Navier-Stokes */
    int flux;           /* 0 Rusanov, 1 HLLC */
    int grad;           /* viscous cell gradients: 0 Green-Gauss, 1 least squares */
} oracle_phys;

/* Boundary condition per face tag (1..7): kind 0 none, 1 Dirichlet state,
 * 2 transmissive (ghost = interior cell average), 3 no-slip adiabatic wall
 * (ghost = interior point state with mirrored velocity), 4 symmetry plane
 * (ghost = mirror image of the interior point state in the face plane; the
 * face's viscous gradient averages the cell's with its mirror image). */
typedef struct {
    int kind[8];
    double state[8][5];
} oracle_bc;

const char* oracle_last_error(void);

/* Geometry, faces, stencils and reconstruction operators.  need[c] != 0 marks
 * cells whose stencils/operators are built (NULL = all). */
int oracle_build(const oracle_mesh_in* in, const oracle_opts* opt, const uint8_t* need,
                 int n_threads, oracle_mesh** out);
void oracle_free(oracle_mesh* m);

/* info[0..10] = n_cell, n_face, K (unknowns), max QPs per face, max faces per
 * cell, max central stencil size, max directional stencil size, min central
 * stencil size, number of boundary faces, number of dropped directional
 * stencils, unknowns of a directional polynomial (3 linear, 9 quadratic) */
int oracle_info(const oracle_mesh* m, int64_t* info);
/* c2f[c*6+lf] = face id (-1 unused), side[c*6+lf] = 0 owner / 1 neighbour */
int oracle_cell_faces(const oracle_mesh* m, int64_t* c2f, int8_t* side);
/* cells[f*2+s] (-1 - tag on boundary side), nq[f], area[f], nrm[f*3], qp[f*QM*3],
 * qw[f*QM], shift[f*3] (neighbour frame = owner frame - shift); QM = max QPs */
int oracle_face_data(const oracle_mesh* m, int64_t* cells, int32_t* nq, double* area, double* nrm,
                     double* qp, double* qw, double* shift);
int oracle_cell_data(const oracle_mesh* m, double* vol, double* cen, double* hbasis);
/* Stencil of one cell: central ids (ncen, up to 128), directional ids [6][32] (ndir[6]),
 * dface[6] = local face of each directional stencil, returns number of directional stencils */
int oracle_stencil(const oracle_mesh* m, int64_t cell, int64_t* central, int32_t* ncen,
                   int64_t* dir, int32_t* ndir, int32_t* dface);
/* Operators of one cell (row-major): Bc[K][ncen], Bd (stencil s's kd x nd[s]
 * block starting at s * kd * 32), O[K][K], Phi[6][QM][K], mean[K]; QM = 16 */
int oracle_operators(const oracle_mesh* m, int64_t cell, double* Bc, double* Bd, double* O,
                     double* Phi, double* mean);
/* Volume quadrature of one cell: up to cap points x[n][3], w[n]; returns n. */
int oracle_cell_quadrature(const oracle_mesh* m, int64_t cell, double* x, double* w, int cap);

/* One reconstruction pass.  U SoA [5][n_cell].  face_state [n_face][2][QM][5]
 * (entries of cells not built stay untouched).  gate_mask (NULL = none):
 * 1 = take the linear central polynomial.  flags[n_cell] (may be NULL):
 * bit0 linear taken, bit1 CWENOZ after failed linear positivity, bit2 first
 * order.  label[n_cell] (may be NULL) = max over variables and stencils of
 * |omega - lambda|. */
int oracle_reconstruct(const oracle_mesh* m, const oracle_phys* ph, const double* U,
                       const uint8_t* gate_mask, double* face_state, uint8_t* flags, double* label);
/* Green-Gauss gradients of (u, v, w, T): gradW [12][n_cell], row = 3*var + dir */
int oracle_gradients(const oracle_mesh* m, const oracle_phys* ph, const oracle_bc* bc,
                     const double* U, double* gradW);
/* Least-squares gradients of (u, v, w, T) over the face neighbours, boundary
 * faces entering through their ghost state at the mirrored centroid; same
 * layout.  The residual path takes this one when ph->grad == 1. */
int oracle_gradients_lsq(const oracle_mesh* m, const oracle_phys* ph, const oracle_bc* bc,
                         const double* U, double* gradW);
/* Face fluxes [n_face][5] (owner -> neighbour, integrated over the face); U
 * (cell averages) supplies the transmissive boundary ghost state */
int oracle_face_flux(const oracle_mesh* m, const oracle_phys* ph, const oracle_bc* bc, const double* U,
                     const double* face_state, const double* gradW, double* face_flux);
/* R [5][n_cell] = -(1/|V|) sum of outward face fluxes */
int oracle_residual(const oracle_mesh* m, const double* face_flux, double* R);
int oracle_dt(const oracle_mesh* m, const oracle_phys* ph, const double* U, double cfl, double* dt);
/* SSP-RK3 stage s: U <- a_s U0 + b_s (U + dt R) */
int oracle_rk_stage(const oracle_mesh* m, int stage, double dt, const double* U0, const double* R,
                    double* U);
/* Five-stage fourth-order SSP-RK stage s (0..4) in Shu-Osher form; W holds
 * u0, u2, u3 and R(u3) as the stages write them ([4][5][n_cell]) */
int oracle_ssp54_stage(const oracle_mesh* m, int stage, double dt, double* W, const double* R, double* U);
/* Mean kinetic energy sum |V| |m|^2/(2 rho) / sum |V| */
int oracle_kinetic_energy(const oracle_mesh* m, const double* U, double* ke);
/* Solenoidal / dilatational dissipation from Green-Gauss velocity gradients */
int oracle_dissipation(const oracle_mesh* m, const oracle_phys* ph, const oracle_bc* bc,
                       const double* U, double* eps_s, double* eps_d);
/* n_steps SSP-RK3 steps in place on U; dt recomputed from U^n each step.
 * ke[n_steps+1], dt_hist[n_steps] may be NULL.  gate_mask applied every stage. */
int oracle_run(const oracle_mesh* m, const oracle_phys* ph, const oracle_bc* bc, double* U,
               double cfl, int n_steps, const uint8_t* gate_mask, double* ke, double* dt_hist);
/* the same with the five-stage fourth-order SSP-RK */
int oracle_run_ssp54(const oracle_mesh* m, const oracle_phys* ph, const oracle_bc* bc, double* U,
                     double cfl, int n_steps, const uint8_t* gate_mask, double* ke, double* dt_hist);

/* Convective numerical flux F(uL, uR; n) of one point (unit normal n) */
int oracle_point_flux(const oracle_phys* ph, const double* uL, const double* uR, const double* n, double* F);

/* Gate features (12 per cell) from cell averages: [n_cell][12] */
int oracle_gate_features(const oracle_mesh* m, const oracle_phys* ph, const double* U, double* feat);

#ifdef __cplusplus
}
#endif
#endif
