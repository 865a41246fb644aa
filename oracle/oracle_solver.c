/* FP64 oracle, part 2: reconstruction, gradients, fluxes, residual, time
 * step, SSP-RK3 and diagnostics.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Each step follows the paper's
 * statement in its order and notation (Sec. 2.2); the readings of the points
 * the paper leaves open are stated where they are used.
 */
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NV 5

/* Positivity thresholds on reconstructed density and pressure (absolute, in
 * the nondimensionalisation rho_ref = 1). */
#define RHO_MIN 1e-10
#define P_MIN 1e-10

static double pressure(const oracle_phys* ph, const double* u) {
    return (ph->gamma - 1.0) * (u[4] - 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0]);
}

/* ------------------------------------------------------- reconstruction */

/* CWENOZ reconstruction of one conserved variable of one cell (Sec. 2.2,
 * eqs. lsq_system, cwenoz_poly, cwenoz_weights).
 *   b_m = U_m - U_i; a_opt = B_c b; a_s = B_s b_s (linear, directional s)
 *   SI_1 = a_opt^T O a_opt; SI_s = a_s^T O_lin a_s
 *   tau = mean_s |SI_1 - SI_s|   (WENO-Z global smoothness measure)
 *   w~_s = lambda_s (1 + tau/(eps + SI_s)), w = w~ / sum w~
 * Blend in the Levy-Puppo-Russo form, p_1 = (p_opt - sum_s lambda_s p_s)/lambda_1,
 * so that w = lambda returns p_opt exactly:
 *   abar = (w_1/lambda_1)(a_opt - sum_s lambda_s a_s) + sum_s w_s a_s.
 * Linear weights: lambda_1 = lambda_c/(lambda_c + n_d), lambda_s = 1/(lambda_c + n_d).
 * Returns max_s |w_s - lambda_s| through *dev. */
static void cwenoz_one_var(const oracle_mesh* m, int64_t c, const double* U, int v, int linear_only,
                           double* abar, double* dev) {
    const oracle_stencil_t* st = m->st[c];
    const oracle_ops_t* op = m->op[c];
    int K = m->K, nd = st->ndir;
    int64_t nc = m->n_cell;
    double ui = U[v * nc + c];
    double a_opt[OR_MAXK];
    for (int k = 0; k < K; ++k) {
        double s = 0;
        for (int j = 0; j < st->ncen; ++j) s += op->Bc[k * st->ncen + j] * (U[v * nc + st->cen[j]] - ui);
        a_opt[k] = s;
    }
    *dev = 0;
    if (linear_only || nd == 0) {
        memcpy(abar, a_opt, sizeof(double) * K);
        return;
    }
    const int kd = m->kd;
    double a_s[OR_MAXF][OR_MAXKD], SI[OR_MAXF + 1];
    for (int s = 0; s < nd; ++s)
        for (int k = 0; k < kd; ++k) {
            double t = 0;
            for (int j = 0; j < st->nd[s]; ++j) t += op->Bd[s][k * st->nd[s] + j] * (U[v * nc + st->dir[s][j]] - ui);
            a_s[s][k] = t;
        }
    /* SI is a sum of squared derivative integrals (non-negative); a rounded
     * quadratic form below zero is rounding, clamped at zero. */
    SI[0] = 0;
    for (int k = 0; k < K; ++k)
        for (int l = 0; l < K; ++l) SI[0] += a_opt[k] * op->O[k * K + l] * a_opt[l];
    SI[0] = fmax(SI[0], 0.0);
    for (int s = 0; s < nd; ++s) {
        double t = 0;
        for (int k = 0; k < kd; ++k)
            for (int l = 0; l < kd; ++l) t += a_s[s][k] * op->O[k * K + l] * a_s[s][l];
        SI[s + 1] = fmax(t, 0.0);
    }
    double tau = 0;
    for (int s = 0; s < nd; ++s) tau += fabs(SI[0] - SI[s + 1]);
    tau /= nd;
    double lam[OR_MAXF + 1], w[OR_MAXF + 1], wsum = 0;
    lam[0] = m->lambda_c / (m->lambda_c + nd);
    for (int s = 1; s <= nd; ++s) lam[s] = 1.0 / (m->lambda_c + nd);
    for (int s = 0; s <= nd; ++s) {
        w[s] = lam[s] * (1.0 + tau / (m->eps + SI[s]));
        wsum += w[s];
    }
    for (int s = 0; s <= nd; ++s) {
        w[s] /= wsum;
        double d = fabs(w[s] - lam[s]);
        if (d > *dev) *dev = d;
    }
    /* p_1 coefficients (LPR), then the blend */
    double p1[OR_MAXK];
    memcpy(p1, a_opt, sizeof(double) * K);
    for (int s = 0; s < nd; ++s)
        for (int k = 0; k < kd; ++k) p1[k] -= lam[s + 1] * a_s[s][k];
    for (int k = 0; k < K; ++k) p1[k] /= lam[0];
    for (int k = 0; k < K; ++k) abar[k] = w[0] * p1[k];
    for (int s = 0; s < nd; ++s)
        for (int k = 0; k < kd; ++k) abar[k] += w[s + 1] * a_s[s][k];
}

/* Evaluate the cell's polynomials at its own face quadrature points
 * (Sec. 2.2, eq. lsq_poly: p = U_i + sum_k a_k phi_k).  Returns 1 if every
 * point has positive density and pressure. */
static int eval_face_states(const oracle_mesh* m, const oracle_phys* ph, int64_t c, const double* U,
                            double abar[NV][OR_MAXK], int first_order, double out[OR_MAXF][OR_QM][NV]) {
    const oracle_ops_t* op = m->op[c];
    int K = m->K, ok = 1;
    for (int lf = 0; lf < or_cell_nfaces(m->type[c]); ++lf) {
        int64_t f = m->c2f[OR_MAXF * c + lf];
        for (int q = 0; q < m->fnq[f]; ++q) {
            const double* phi = op->Phi + (size_t)(lf * OR_QM + q) * K;
            for (int v = 0; v < NV; ++v) {
                double s = U[v * m->n_cell + c];
                if (!first_order)
                    for (int k = 0; k < K; ++k) s += abar[v][k] * phi[k];
                out[lf][q][v] = s;
            }
            if (!(out[lf][q][0] > RHO_MIN) || !(pressure(ph, out[lf][q]) > P_MIN)) ok = 0;
        }
    }
    return ok;
}

int oracle_reconstruct(const oracle_mesh* m, const oracle_phys* ph, const double* U, const uint8_t* gate_mask,
                       double* face_state, uint8_t* flags, double* label) {
    int64_t nc = m->n_cell;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < nc; ++c) {
        if (!m->need[c]) continue;
        double abar[NV][OR_MAXK], st[OR_MAXF][OR_QM][NV], dev, maxdev = 0;
        uint8_t fl = 0;
        int linear = gate_mask ? (gate_mask[c] != 0) : 0;
        for (int v = 0; v < NV; ++v) {
            cwenoz_one_var(m, c, U, v, linear, abar[v], &dev);
            if (dev > maxdev) maxdev = dev;
        }
        if (linear) fl |= 1;
        int ok = eval_face_states(m, ph, c, U, abar, 0, st);
        if (!ok && linear) {
            /* fallback chain: linear -> full CWENOZ -> first order */
            fl |= 2;
            for (int v = 0; v < NV; ++v) cwenoz_one_var(m, c, U, v, 0, abar[v], &dev);
            ok = eval_face_states(m, ph, c, U, abar, 0, st);
        }
        if (!ok) {
            fl |= 4;
            eval_face_states(m, ph, c, U, abar, 1, st);
        }
        for (int lf = 0; lf < or_cell_nfaces(m->type[c]); ++lf) {
            int64_t f = m->c2f[OR_MAXF * c + lf];
            int side = m->c2s[OR_MAXF * c + lf];
            for (int q = 0; q < m->fnq[f]; ++q)
                for (int v = 0; v < NV; ++v) face_state[(((size_t)f * 2 + side) * OR_QM + q) * NV + v] = st[lf][q][v];
        }
        if (flags) flags[c] = fl;
        if (label) label[c] = maxdev;
    }
    return 0;
}

/* ------------------------------------------------------------- physics */

/* Primitive viscous variables W = (u, v, w, T) with the nondimensional
 * temperature T = gamma M^2 p / rho (rho_ref = u_ref = L = 1). */
static void prim_W(const oracle_phys* ph, const double* u, double* W) {
    W[0] = u[1] / u[0];
    W[1] = u[2] / u[0];
    W[2] = u[3] / u[0];
    W[3] = ph->gamma * ph->mach * ph->mach * pressure(ph, u) / u[0];
}

/* Ghost state across a boundary face (tag kinds in oracle.h): Dirichlet takes
 * the prescribed state; the no-slip wall mirrors the full velocity of the
 * interior point state `in`; the symmetry plane is the mirror image of `in`
 * in the face plane (unit normal n): density and energy kept, momentum
 * reflected by M = I - 2 n n^T; transmissive (zero-gradient) outflow copies
 * the interior cell's average `avg` (zeroth-order extrapolation: copying the
 * reconstructed point value instead feeds a one-sided extrapolation back
 * into the boundary cell). */
static void ghost_state(const oracle_bc* bc, int tag, const double* in, const double* avg, const double* n,
                        double* out) {
    int kind = bc ? bc->kind[tag] : 2;
    if (kind == 1) {
        memcpy(out, bc->state[tag], sizeof(double) * NV);
    } else if (kind == 3) {
        out[0] = in[0];
        out[1] = -in[1];
        out[2] = -in[2];
        out[3] = -in[3];
        out[4] = in[4];
    } else if (kind == 4) {
        out[0] = in[0];
        for (int a = 0; a < 3; ++a) {
            out[1 + a] = 0.0;
            for (int b = 0; b < 3; ++b) out[1 + a] += ((a == b ? 1.0 : 0.0) - 2.0 * n[a] * n[b]) * in[1 + b];
        }
        out[4] = in[4];
    } else {
        memcpy(out, avg, sizeof(double) * NV);
    }
}

static void euler_flux_n(const oracle_phys* ph, const double* u, const double* n, double* F) {
    double rho = u[0], vx = u[1] / rho, vy = u[2] / rho, vz = u[3] / rho;
    double p = pressure(ph, u), un = vx * n[0] + vy * n[1] + vz * n[2];
    F[0] = rho * un;
    F[1] = u[1] * un + p * n[0];
    F[2] = u[2] * un + p * n[1];
    F[3] = u[3] * un + p * n[2];
    F[4] = (u[4] + p) * un;
}

/* Rusanov (local Lax-Friedrichs) flux, s = max(|u_nL| + c_L, |u_nR| + c_R). */
static void rusanov(const oracle_phys* ph, const double* L, const double* R, const double* n, double* F) {
    double FL[NV], FR[NV];
    euler_flux_n(ph, L, n, FL);
    euler_flux_n(ph, R, n, FR);
    double unL = (L[1] * n[0] + L[2] * n[1] + L[3] * n[2]) / L[0];
    double unR = (R[1] * n[0] + R[2] * n[1] + R[3] * n[2]) / R[0];
    double cL = sqrt(ph->gamma * pressure(ph, L) / L[0]);
    double cR = sqrt(ph->gamma * pressure(ph, R) / R[0]);
    double s = fmax(fabs(unL) + cL, fabs(unR) + cR);
    for (int v = 0; v < NV; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * s * (R[v] - L[v]);
}

/* HLLC flux of Toro, Spruce & Speares with Davis wave-speed estimates
 * S_L = min(u_nL - c_L, u_nR - c_R), S_R = max(u_nL + c_L, u_nR + c_R);
 * star states in rotation-free form.  S* >= 0 takes the left star state. */
static void hllc(const oracle_phys* ph, const double* L, const double* R, const double* n, double* F) {
    double rL = L[0], rR = R[0];
    double unL = (L[1] * n[0] + L[2] * n[1] + L[3] * n[2]) / rL;
    double unR = (R[1] * n[0] + R[2] * n[1] + R[3] * n[2]) / rR;
    double pL = pressure(ph, L), pR = pressure(ph, R);
    double cL = sqrt(ph->gamma * pL / rL), cR = sqrt(ph->gamma * pR / rR);
    double SL = fmin(unL - cL, unR - cR), SR = fmax(unL + cL, unR + cR);
    double Ss = (pR - pL + rL * unL * (SL - unL) - rR * unR * (SR - unR)) / (rL * (SL - unL) - rR * (SR - unR));
    double FK[NV];
    if (SL >= 0) {
        euler_flux_n(ph, L, n, F);
        return;
    }
    if (SR <= 0) {
        euler_flux_n(ph, R, n, F);
        return;
    }
    const double* K = Ss >= 0 ? L : R;
    double SK = Ss >= 0 ? SL : SR, unK = Ss >= 0 ? unL : unR, pK = Ss >= 0 ? pL : pR;
    euler_flux_n(ph, K, n, FK);
    double chi = (SK - unK) / (SK - Ss);
    double rho = K[0];
    double Us[NV];
    Us[0] = rho * chi;
    for (int a = 0; a < 3; ++a) Us[1 + a] = rho * chi * (K[1 + a] / rho + (Ss - unK) * n[a]);
    Us[4] = rho * chi * (K[4] / rho + (Ss - unK) * (Ss + pK / (rho * (SK - unK))));
    for (int v = 0; v < NV; ++v) F[v] = FK[v] + SK * (Us[v] - K[v]);
}

/* ------------------------------------------------------------ gradients */

/* Green-Gauss cell gradients of W = (u, v, w, T) from cell averages, face
 * value the arithmetic mean of the two cells (boundary: of the cell and its
 * ghost). */
int oracle_gradients(const oracle_mesh* m, const oracle_phys* ph, const oracle_bc* bc, const double* U,
                     double* gradW) {
    int64_t nc = m->n_cell;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        double ui[NV], Wi[4], g[12] = {0};
        for (int v = 0; v < NV; ++v) ui[v] = U[v * nc + c];
        prim_W(ph, ui, Wi);
        for (int lf = 0; lf < or_cell_nfaces(m->type[c]); ++lf) {
            int64_t f = m->c2f[OR_MAXF * c + lf];
            int side = m->c2s[OR_MAXF * c + lf];
            double sgn = side ? -1.0 : 1.0, n[3];
            for (int a = 0; a < 3; ++a) n[a] = m->fnrm[3 * f + a];
            int64_t other = m->fcell[2 * f + (1 - side)];
            double uo[NV], Wo[4];
            if (other >= 0) {
                for (int v = 0; v < NV; ++v) uo[v] = U[v * nc + other];
            } else {
                ghost_state(bc, (int)(-1 - other), ui, ui, n, uo);
            }
            prim_W(ph, uo, Wo);
            for (int var = 0; var < 4; ++var)
                for (int a = 0; a < 3; ++a) g[3 * var + a] += 0.5 * (Wi[var] + Wo[var]) * sgn * n[a] * m->farea[f];
        }
        for (int k = 0; k < 12; ++k) gradW[k * nc + c] = g[k] / m->vol[c];
    }
    return 0;
}

/* Least-squares cell gradients of W = (u, v, w, T) (Sec. 2.2:
 * the viscous terms take least-squares gradients with boundary-condition
 * constraints).  Reading of what the paper leaves open: a linear fit
 *     min_g  sum_j w_j (W_j - W_i - g . d_j)^2,   w_j = 1 / |d_j|^2,
 * over the face neighbours j, with d_j the offset from c_i to the image of
 * c_j next to cell i (periodic seams included).  A boundary face enters as
 * its ghost state (the same ghost as above) placed at the mirror image of c_i
 * in the face plane, d = 2 ((x_f - c_i) . n) n: the no-slip wall's mirrored
 * velocity puts u = 0 on the wall, the wall's temperature and the
 * transmissive ghost give zero normal derivative, a Dirichlet ghost imposes
 * its state.  Solved per cell from the 3x3 normal equations by Cramer's rule. */
static double det3(const double A[3][3]) {
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

int oracle_gradients_lsq(const oracle_mesh* m, const oracle_phys* ph, const oracle_bc* bc, const double* U,
                         double* gradW) {
    int64_t nc = m->n_cell;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t c = 0; c < nc; ++c) {
        double ui[NV], Wi[4], M[3][3] = {{0}}, rhs[4][3] = {{0}};
        for (int v = 0; v < NV; ++v) ui[v] = U[v * nc + c];
        prim_W(ph, ui, Wi);
        for (int lf = 0; lf < or_cell_nfaces(m->type[c]); ++lf) {
            int64_t f = m->c2f[OR_MAXF * c + lf];
            int side = m->c2s[OR_MAXF * c + lf];
            int64_t other = m->fcell[2 * f + (1 - side)];
            double uo[NV], Wo[4], d[3];
            if (other >= 0) {
                /* the neighbour's image next to c: owner frame = neighbour frame + shift */
                double sh = side ? -1.0 : 1.0;
                for (int a = 0; a < 3; ++a) d[a] = m->cen[3 * other + a] + sh * m->fshift[3 * f + a] - m->cen[3 * c + a];
                for (int v = 0; v < NV; ++v) uo[v] = U[v * nc + other];
            } else {
                double dn = 0;
                for (int a = 0; a < 3; ++a) dn += (m->fcen[3 * f + a] - m->cen[3 * c + a]) * m->fnrm[3 * f + a];
                for (int a = 0; a < 3; ++a) d[a] = 2.0 * dn * m->fnrm[3 * f + a];
                ghost_state(bc, (int)(-1 - other), ui, ui, m->fnrm + 3 * f, uo);
            }
            prim_W(ph, uo, Wo);
            double w = 1.0 / (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) M[a][b] += w * d[a] * d[b];
            for (int var = 0; var < 4; ++var)
                for (int a = 0; a < 3; ++a) rhs[var][a] += w * d[a] * (Wo[var] - Wi[var]);
        }
        double det = det3(M);
        if (!(fabs(det) > 0)) {
            bad = 1;
            continue;
        }
        for (int var = 0; var < 4; ++var)
            for (int a = 0; a < 3; ++a) {
                /* Cramer: replace column a of M by the right-hand side */
                double A[3][3];
                for (int r = 0; r < 3; ++r)
                    for (int k = 0; k < 3; ++k) A[r][k] = k == a ? rhs[var][r] : M[r][k];
                gradW[(3 * var + a) * nc + c] = det3(A) / det;
            }
    }
    return bad ? or_fail(-1, "singular least-squares gradient system") : 0;
}

/* Viscous-gradient choice of the physics options: Green-Gauss or least squares. */
static int cell_gradients(const oracle_mesh* m, const oracle_phys* ph, const oracle_bc* bc, const double* U,
                          double* gradW) {
    return ph->grad == 1 ? oracle_gradients_lsq(m, ph, bc, U, gradW) : oracle_gradients(m, ph, bc, U, gradW);
}

/* ------------------------------------------------------------ face flux */

/* Gradient of the mirror image of a flow in the plane with unit normal n:
 * with M = I - 2 n n^T the mirrored velocity field u'(x) = M u(Mx) has
 * gradient M G M (G_ij = du_i/dx_j), the mirrored temperature gradient M g_T.
 * A symmetry face averages the cell's gradient with this one. */
static void mirror_gradient(const double* g, const double* n, double* gm) {
    double M[3][3], MG[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) M[a][b] = (a == b ? 1.0 : 0.0) - 2.0 * n[a] * n[b];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            MG[i][j] = 0.0;
            for (int k = 0; k < 3; ++k) MG[i][j] += M[i][k] * g[3 * k + j];
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            gm[3 * i + j] = 0.0;
            for (int k = 0; k < 3; ++k) gm[3 * i + j] += MG[i][k] * M[k][j];
        }
    for (int j = 0; j < 3; ++j) {
        gm[9 + j] = 0.0;
        for (int k = 0; k < 3; ++k) gm[9 + j] += M[j][k] * g[9 + k];
    }
}

/* Viscous flux F_v . n at one quadrature point (Newtonian stress with
 * Stokes' hypothesis, Fourier heat flux).  Reading of the closure the paper
 * leaves open: mu = 1/Re constant, kappa = mu / ((gamma-1) M^2 Pr).
 * Interface gradient (Sec. 2.2, eq. viscous_gradient_penalty) with
 * alpha = 4/3, applied to W, U_L/U_R the two reconstructed point states. */
static void viscous_flux(const oracle_phys* ph, const double* uL, const double* uR, const double* gL,
                         const double* gR, const double* n, double Lint, double* Fv) {
    double WL[4], WR[4], Wf[4], G[4][3];
    prim_W(ph, uL, WL);
    prim_W(ph, uR, WR);
    const double alpha = 4.0 / 3.0;
    for (int var = 0; var < 4; ++var) {
        Wf[var] = 0.5 * (WL[var] + WR[var]);
        for (int a = 0; a < 3; ++a)
            G[var][a] = 0.5 * (gL[3 * var + a] + gR[3 * var + a]) + alpha / Lint * (WR[var] - WL[var]) * n[a];
    }
    double mu = 1.0 / ph->reynolds;
    double kappa = mu / ((ph->gamma - 1.0) * ph->mach * ph->mach * ph->prandtl);
    double div = G[0][0] + G[1][1] + G[2][2];
    double tau[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) tau[i][j] = mu * (G[i][j] + G[j][i] - (i == j ? 2.0 / 3.0 * div : 0.0));
    Fv[0] = 0;
    double e = 0;
    for (int i = 0; i < 3; ++i) {
        double t = 0;
        for (int j = 0; j < 3; ++j) t += tau[i][j] * n[j];
        Fv[1 + i] = t;
        e += Wf[i] * t;
    }
    for (int j = 0; j < 3; ++j) e += kappa * G[3][j] * n[j];
    Fv[4] = e;
}

/* F_f = |S_f| sum_q w_q (F_c(U_L, U_R; n) - F_v) (Sec. 2.2, eq. fv_update). */
int oracle_face_flux(const oracle_mesh* m, const oracle_phys* ph, const oracle_bc* bc, const double* U,
                     const double* face_state, const double* gradW, double* face_flux) {
    int64_t nf = m->n_face, nc = m->n_cell;
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < nf; ++f) {
        int64_t cL = m->fcell[2 * f], cR = m->fcell[2 * f + 1];
        const double* n = m->fnrm + 3 * f;
        double acc[NV] = {0}, uavg[NV];
        for (int v = 0; v < NV; ++v) uavg[v] = U[v * nc + cL];
        double gL[12], gR[12], Lint = 1.0;
        if (ph->viscous) {
            for (int k = 0; k < 12; ++k) gL[k] = gradW[k * nc + cL];
            if (cR >= 0) {
                for (int k = 0; k < 12; ++k) gR[k] = gradW[k * nc + cR];
                double d[3];
                for (int a = 0; a < 3; ++a) d[a] = m->cen[3 * cR + a] + m->fshift[3 * f + a] - m->cen[3 * cL + a];
                Lint = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            } else {
                if (bc && bc->kind[-1 - cR] == 4) {
                    mirror_gradient(gL, n, gR);
                } else {
                    memcpy(gR, gL, sizeof gL);
                }
                double d = 0;
                for (int a = 0; a < 3; ++a) d += (m->fcen[3 * f + a] - m->cen[3 * cL + a]) * n[a];
                Lint = 2.0 * fabs(d);
            }
        }
        for (int q = 0; q < m->fnq[f]; ++q) {
            const double* uL = face_state + ((size_t)f * 2 * OR_QM + q) * NV;
            double uRb[NV];
            const double* uR;
            if (cR >= 0) {
                uR = face_state + (((size_t)f * 2 + 1) * OR_QM + q) * NV;
            } else {
                ghost_state(bc, (int)(-1 - cR), uL, uavg, n, uRb);
                uR = uRb;
            }
            double F[NV];
            if (ph->flux == 1)
                hllc(ph, uL, uR, n, F);
            else
                rusanov(ph, uL, uR, n, F);
            if (ph->viscous) {
                double Fv[NV];
                viscous_flux(ph, uL, uR, gL, gR, n, Lint, Fv);
                for (int v = 0; v < NV; ++v) F[v] -= Fv[v];
            }
            double w = m->fqw[(size_t)f * OR_QM + q];
            for (int v = 0; v < NV; ++v) acc[v] += w * F[v];
        }
        for (int v = 0; v < NV; ++v) face_flux[f * NV + v] = m->farea[f] * acc[v];
    }
    return 0;
}

/* ------------------------------------------------------------- residual */

/* R_i = -(1/|V_i|) sum_f s_if F_f, faces in local order, s = +1 for the
 * owner, -1 for the neighbour (Sec. 2.2, eq. fv_update). */
int oracle_residual(const oracle_mesh* m, const double* face_flux, double* R) {
    int64_t nc = m->n_cell;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        double acc[NV] = {0};
        for (int lf = 0; lf < or_cell_nfaces(m->type[c]); ++lf) {
            int64_t f = m->c2f[OR_MAXF * c + lf];
            double s = m->c2s[OR_MAXF * c + lf] ? -1.0 : 1.0;
            for (int v = 0; v < NV; ++v) acc[v] += s * face_flux[f * NV + v];
        }
        for (int v = 0; v < NV; ++v) R[v * nc + c] = -acc[v] / m->vol[c];
    }
    return 0;
}

/* --------------------------------------------------------- time stepping */

/* dt = CFL min_i h_i / (|u_i| + c_i), h_i = 6 |V_i| / sum_f |S_f|; with
 * viscosity also dt <= CFL min_i rho_i h_i^2 / (2 mu max(4/3, gamma/Pr)). */
int oracle_dt(const oracle_mesh* m, const oracle_phys* ph, const double* U, double cfl, double* dt) {
    int64_t nc = m->n_cell;
    double best = INFINITY;
    for (int64_t c = 0; c < nc; ++c) {
        double u[NV];
        for (int v = 0; v < NV; ++v) u[v] = U[v * nc + c];
        double sp = sqrt(u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0];
        double cs = sqrt(ph->gamma * pressure(ph, u) / u[0]);
        double h = m->hdt[c];
        double t = h / (sp + cs);
        if (ph->viscous) {
            double mu = 1.0 / ph->reynolds;
            double k = fmax(4.0 / 3.0, ph->gamma / ph->prandtl);
            double tv = u[0] * h * h / (2.0 * mu * k);
            if (tv < t) t = tv;
        }
        if (!(t > 0)) return or_fail(-7, "invalid time step at cell %lld", (long long)c);
        if (t < best) best = t;
    }
    *dt = cfl * best;
    return 0;
}

/* Shu-Osher SSP-RK3: U1 = U^n + dt R(U^n); U2 = 3/4 U^n + 1/4 (U1 + dt R(U1));
 * U^{n+1} = 1/3 U^n + 2/3 (U2 + dt R(U2)). */
int oracle_rk_stage(const oracle_mesh* m, int stage, double dt, const double* U0, const double* R, double* U) {
    static const double A[3] = {0.0, 0.75, 1.0 / 3.0}, B[3] = {1.0, 0.25, 2.0 / 3.0};
    if (stage < 0 || stage > 2) return or_fail(-1, "stage %d", stage);
    int64_t n = NV * m->n_cell;
    for (int64_t k = 0; k < n; ++k) U[k] = A[stage] * U0[k] + B[stage] * (U[k] + dt * R[k]);
    return 0;
}

/* Five-stage fourth-order SSP Runge-Kutta (Spiteri & Ruuth 2002, the
 * integrator family the paper uses, Sec. 2.2), Shu-Osher form with L = R:
 *   u1 = u0 + b10 dt L(u0)
 *   u2 = a20 u0 + a21 u1 + b21 dt L(u1)
 *   u3 = a30 u0 + a32 u2 + b32 dt L(u2)
 *   u4 = a40 u0 + a43 u3 + b43 dt L(u3)
 *   u5 = a52 u2 + a53 u3 + b53 dt L(u3) + a54 u4 + b54 dt L(u4)
 * Stage s takes R = L(U) of the current U; W holds u0, u2, u3 and L(u3)
 * (four blocks of NV n_cell values), written as the stages reach them. */
int oracle_ssp54_stage(const oracle_mesh* m, int stage, double dt, double* W, const double* R, double* U) {
    static const double b10 = 0.391752226571890;
    static const double a20 = 0.444370493651235, a21 = 0.555629506348765, b21 = 0.368410593050371;
    static const double a30 = 0.620101851488403, a32 = 0.379898148511597, b32 = 0.251891774271694;
    static const double a40 = 0.178079954393132, a43 = 0.821920045606868, b43 = 0.544974750228521;
    static const double a52 = 0.517231671970585, a53 = 0.096059710526147, b53 = 0.063692468666290;
    static const double a54 = 0.386708617503269, b54 = 0.226007483236906;
    if (stage < 0 || stage > 4) return or_fail(-1, "stage %d", stage);
    int64_t n = NV * m->n_cell;
    double *u0 = W, *u2 = W + n, *u3 = W + 2 * n, *L3 = W + 3 * n;
    for (int64_t k = 0; k < n; ++k) {
        double u = U[k], r = R[k];
        switch (stage) {
            case 0: u0[k] = u; U[k] = u + b10 * dt * r; break;
            case 1: U[k] = a20 * u0[k] + a21 * u + b21 * dt * r; u2[k] = U[k]; break;
            case 2: U[k] = a30 * u0[k] + a32 * u + b32 * dt * r; u3[k] = U[k]; break;
            case 3: L3[k] = r; U[k] = a40 * u0[k] + a43 * u + b43 * dt * r; break;
            default: U[k] = a52 * u2[k] + a53 * u3[k] + b53 * dt * L3[k] + a54 * u + b54 * dt * r; break;
        }
    }
    return 0;
}

int oracle_kinetic_energy(const oracle_mesh* m, const double* U, double* ke) {
    int64_t nc = m->n_cell;
    double s = 0, vs = 0;
    for (int64_t c = 0; c < nc; ++c) {
        double r = U[c], mx = U[nc + c], my = U[2 * nc + c], mz = U[3 * nc + c];
        s += m->vol[c] * 0.5 * (mx * mx + my * my + mz * mz) / r;
        vs += m->vol[c];
    }
    *ke = s / vs;
    return 0;
}

/* eps_s = (mu/|Omega|) sum |V| |curl u|^2, eps_d = (4 mu / 3|Omega|) sum |V| (div u)^2,
 * from Green-Gauss gradients (unit reference density). */
int oracle_dissipation(const oracle_mesh* m, const oracle_phys* ph, const oracle_bc* bc, const double* U,
                       double* eps_s, double* eps_d) {
    int64_t nc = m->n_cell;
    double* g = malloc(sizeof(double) * 12 * nc);
    oracle_gradients(m, ph, bc, U, g);
    double mu = 1.0 / ph->reynolds, ss = 0, sd = 0, vs = 0;
    for (int64_t c = 0; c < nc; ++c) {
#define G(var, a) g[(3 * (var) + (a)) * nc + c]
        double wx = G(2, 1) - G(1, 2), wy = G(0, 2) - G(2, 0), wz = G(1, 0) - G(0, 1);
        double dv = G(0, 0) + G(1, 1) + G(2, 2);
#undef G
        ss += m->vol[c] * (wx * wx + wy * wy + wz * wz);
        sd += m->vol[c] * dv * dv;
        vs += m->vol[c];
    }
    free(g);
    *eps_s = mu * ss / vs;
    *eps_d = 4.0 * mu / 3.0 * sd / vs;
    return 0;
}

static int eval_rhs(const oracle_mesh* m, const oracle_phys* ph, const oracle_bc* bc, const double* U,
                    const uint8_t* gate_mask, double* fs, double* gw, double* ff, double* R) {
    int rc = oracle_reconstruct(m, ph, U, gate_mask, fs, NULL, NULL);
    if (rc) return rc;
    if (ph->viscous) {
        rc = cell_gradients(m, ph, bc, U, gw);
        if (rc) return rc;
    }
    oracle_face_flux(m, ph, bc, U, fs, ph->viscous ? gw : NULL, ff);
    return oracle_residual(m, ff, R);
}

static int run_steps(const oracle_mesh* m, const oracle_phys* ph, const oracle_bc* bc, double* U, double cfl,
                     int n_steps, const uint8_t* gate_mask, double* ke, double* dt_hist, int ssp54);

int oracle_run(const oracle_mesh* m, const oracle_phys* ph, const oracle_bc* bc, double* U, double cfl,
               int n_steps, const uint8_t* gate_mask, double* ke, double* dt_hist) {
    return run_steps(m, ph, bc, U, cfl, n_steps, gate_mask, ke, dt_hist, 0);
}

int oracle_run_ssp54(const oracle_mesh* m, const oracle_phys* ph, const oracle_bc* bc, double* U, double cfl,
                     int n_steps, const uint8_t* gate_mask, double* ke, double* dt_hist) {
    return run_steps(m, ph, bc, U, cfl, n_steps, gate_mask, ke, dt_hist, 1);
}

static int run_steps(const oracle_mesh* m, const oracle_phys* ph, const oracle_bc* bc, double* U, double cfl,
                     int n_steps, const uint8_t* gate_mask, double* ke, double* dt_hist, int ssp54) {
    int64_t nc = m->n_cell, nf = m->n_face;
    for (int64_t c = 0; c < nc; ++c)
        if (!m->need[c]) return or_fail(-1, "oracle_run needs every cell built");
    double* U0 = malloc(sizeof(double) * NV * nc * (ssp54 ? 4 : 1));
    double* R = malloc(sizeof(double) * NV * nc);
    double* fs = calloc((size_t)nf * 2 * OR_QM * NV, sizeof(double));
    double* ff = malloc(sizeof(double) * NV * nf);
    double* gw = ph->viscous ? malloc(sizeof(double) * 12 * nc) : NULL;
    int rc = 0;
    if (ke) oracle_kinetic_energy(m, U, &ke[0]);
    for (int n = 0; n < n_steps && !rc; ++n) {
        double dt;
        rc = oracle_dt(m, ph, U, cfl, &dt);
        if (rc) break;
        if (dt_hist) dt_hist[n] = dt;
        if (!ssp54) memcpy(U0, U, sizeof(double) * NV * nc);
        for (int s = 0; s < (ssp54 ? 5 : 3) && !rc; ++s) {
            rc = eval_rhs(m, ph, bc, U, gate_mask, fs, gw, ff, R);
            if (!rc) rc = ssp54 ? oracle_ssp54_stage(m, s, dt, U0, R, U) : oracle_rk_stage(m, s, dt, U0, R, U);
        }
        if (ke) oracle_kinetic_energy(m, U, &ke[n + 1]);
    }
    free(U0);
    free(R);
    free(fs);
    free(ff);
    free(gw);
    return rc;
}

/* ------------------------------------------------------------ gate features */

/* Twelve features of a cell for the troubled-cell gate, for v in (rho, rho E):
 *  (1) max and (2) mean over the central stencil of |v_m - v_i| / |v_i|;
 *  (3) h |grad p_opt| / |v_i| with the central polynomial's gradient at the centroid;
 *  (4-6) max, mean, min over face neighbours j of
 *        |v_j - v_i - grad p_opt . (c_j - c_i)| / (|v_j - v_i| + h |grad p_opt| + 1e-12 |v_i|).
 * Each feature is mapped through log(1e-12 + x). */
int oracle_gate_features(const oracle_mesh* m, const oracle_phys* ph, const double* U, double* feat) {
    (void)ph;
    int64_t nc = m->n_cell;
    const int vars[2] = {0, 4};
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < nc; ++c) {
        if (!m->need[c]) continue;
        const oracle_stencil_t* st = m->st[c];
        const oracle_ops_t* op = m->op[c];
        double h = m->hbasis[c];
        for (int t = 0; t < 2; ++t) {
            int v = vars[t];
            double ui = U[v * nc + c], au = fabs(ui);
            double mx = 0, mean = 0;
            double a[OR_MAXK];
            for (int k = 0; k < m->K; ++k) {
                double s = 0;
                for (int j = 0; j < st->ncen; ++j) s += op->Bc[k * st->ncen + j] * (U[v * nc + st->cen[j]] - ui);
                a[k] = s;
            }
            for (int j = 0; j < st->ncen; ++j) {
                double d = fabs(U[v * nc + st->cen[j]] - ui) / au;
                if (d > mx) mx = d;
                mean += d;
            }
            mean /= st->ncen;
            /* gradient of p_opt at the centroid: only the linear monomials contribute */
            double gx = a[0] / h, gy = a[1] / h, gz = a[2] / h;
            double gn = sqrt(gx * gx + gy * gy + gz * gz);
            double dmax = 0, dmean = 0, dmin = INFINITY;
            int cnt = 0;
            for (int lf = 0; lf < or_cell_nfaces(m->type[c]); ++lf) {
                int64_t f = m->c2f[OR_MAXF * c + lf];
                int side = m->c2s[OR_MAXF * c + lf];
                int64_t j = m->fcell[2 * f + (1 - side)];
                if (j < 0) continue;
                double d[3];
                for (int k = 0; k < 3; ++k) {
                    d[k] = m->cen[3 * j + k] - m->cen[3 * c + k];
                    if (m->period[k] > 0) d[k] -= m->period[k] * nearbyint(d[k] / m->period[k]);
                }
                double uj = U[v * nc + j];
                double num = fabs(uj - ui - (gx * d[0] + gy * d[1] + gz * d[2]));
                double den = fabs(uj - ui) + h * gn + 1e-12 * au;
                double r = num / den;
                if (r > dmax) dmax = r;
                if (r < dmin) dmin = r;
                dmean += r;
                ++cnt;
            }
            dmean /= cnt;
            double* o = feat + (size_t)c * 12 + 6 * t;
            o[0] = log(1e-12 + mx);
            o[1] = log(1e-12 + mean);
            o[2] = log(1e-12 + h * gn / au);
            o[3] = log(1e-12 + dmax);
            o[4] = log(1e-12 + dmean);
            o[5] = log(1e-12 + dmin);
        }
    }
    return 0;
}

/* Convective flux of one point state pair (for the flux pins). */
int oracle_point_flux(const oracle_phys* ph, const double* uL, const double* uR, const double* n, double* F) {
    if (ph->flux == 1)
        hllc(ph, uL, uR, n, F);
    else
        rusanov(ph, uL, uR, n, F);
    return 0;
}
