/* FP64 oracle, part 1: geometry, faces, quadrature, basis, stencils and
 * least-squares reconstruction operators.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain loops, written for
 * checkability rather than speed.
 *
 * Method references are to the paper "Towards Heterogeneous Exascale CFD with
 * a Single Fortran Code Base" (UCNS3D v4): Sec. 2.2, equations lsq_poly,
 * lsq_system, cwenoz_poly, cwenoz_weights, viscous_gradient_penalty,
 * fv_update.  Where the paper is silent the reading used is stated inline.
 */
#include "oracle_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static __thread char g_err[512];

const char* oracle_last_error(void) { return g_err; }

int or_fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

/* ------------------------------------------------------------------ tables */

/* Local faces of each cell type; vertex order gives the outward normal by the
 * right-hand rule.  Tet and hex use VTK vertex numbering. */
static const int TET_F[4][4] = {{1, 2, 3, -1}, {0, 3, 2, -1}, {0, 1, 3, -1}, {0, 2, 1, -1}};
static const int HEX_F[6][4] = {{0, 4, 7, 3}, {1, 2, 6, 5}, {0, 1, 5, 4},
                                {3, 7, 6, 2}, {0, 3, 2, 1}, {4, 5, 6, 7}};
static const int PRI_F[5][4] = {{0, 2, 1, -1}, {3, 4, 5, -1}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}};
static const int PYR_F[5][4] = {{0, 3, 2, 1}, {0, 1, 4, -1}, {1, 2, 4, -1}, {2, 3, 4, -1}, {3, 0, 4, -1}};

int or_cell_nfaces(int type) {
    switch (type) {
    case 4: return 4;
    case 5: return 5;
    case 6: return 5;
    case 8: return 6;
    }
    return -1;
}

const int* or_face_verts(int type, int lf, int* nv) {
    const int* row;
    switch (type) {
    case 4: row = TET_F[lf]; break;
    case 5: row = PYR_F[lf]; break;
    case 6: row = PRI_F[lf]; break;
    default: row = HEX_F[lf]; break;
    }
    *nv = row[3] < 0 ? 3 : 4;
    return row;
}

/* Number of polynomial coefficients of degree <= r in 3-D including the
 * constant: K(r,3) = (r+1)(r+2)(r+3)/6 (Sec. 2.2, eq. lsq_poly). */
int or_K(int r) { return (r + 1) * (r + 2) * (r + 3) / 6; }

/* Graded-lexicographic exponents of the monomials of degree 1..r. */
static void monomial_exponents(int r, int e[][3]) {
    int k = 0;
    for (int d = 1; d <= r; ++d)
        for (int a = d; a >= 0; --a)
            for (int b = d - a; b >= 0; --b) {
                e[k][0] = a;
                e[k][1] = b;
                e[k][2] = d - a - b;
                ++k;
            }
}

static double ipow(double x, int n) {
    double r = 1.0;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
}

static void gauss_legendre01(int n, double* x, double* w) {
    /* Newton iteration on P_n for the nodes on [-1,1], then map to [0,1]. */
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int j = 0; j < n; ++j) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * j + 1.0) * z * p1 - j * p2) / (j + 1.0);
            }
            pp = n * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / pp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * pp * pp);
    }
}

/* ----------------------------------------------------------- vector helpers */

static void sub3(const double* a, const double* b, double* c) {
    c[0] = a[0] - b[0];
    c[1] = a[1] - b[1];
    c[2] = a[2] - b[2];
}
static void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double norm3(const double* a) { return sqrt(dot3(a, a)); }

/* Periodic minimum-image wrap of a displacement. */
static void min_image(const oracle_mesh* m, double* d) {
    for (int a = 0; a < 3; ++a)
        if (m->period[a] > 0.0) d[a] -= m->period[a] * nearbyint(d[a] / m->period[a]);
}

/* Vertex coordinates of a cell, each taken as the periodic image nearest the
 * cell's first vertex. */
int or_cell_coords(const oracle_mesh* m, int64_t c, double X[8][3]) {
    int64_t p0 = m->cell_ptr[c], nv = m->cell_ptr[c + 1] - p0;
    const double* x0 = m->xyz + 3 * m->cell_vtx[p0];
    for (int k = 0; k < nv; ++k) {
        const double* x = m->xyz + 3 * m->cell_vtx[p0 + k];
        for (int a = 0; a < 3; ++a) {
            double v = x[a];
            if (m->period[a] > 0.0) v -= m->period[a] * nearbyint((x[a] - x0[a]) / m->period[a]);
            X[k][a] = v;
        }
    }
    return (int)nv;
}

/* Sub-tetrahedra of a cell: apex at the vertex average, bases on the face
 * triangles (a quadrilateral face is fanned into 4 triangles around its
 * vertex average).  Returns the count; T[t][4][3]. */
static int cell_subtets(const oracle_mesh* m, int64_t c, double T[24][4][3]) {
    double X[8][3];
    int type = m->type[c];
    int nv = or_cell_coords(m, c, X);
    double ctr[3] = {0, 0, 0};
    for (int k = 0; k < nv; ++k)
        for (int a = 0; a < 3; ++a) ctr[a] += X[k][a] / nv;
    int nt = 0, nf = or_cell_nfaces(type);
    for (int lf = 0; lf < nf; ++lf) {
        int fnv;
        const int* fv = or_face_verts(type, lf, &fnv);
        if (fnv == 3) {
            memcpy(T[nt][0], ctr, sizeof ctr);
            for (int j = 0; j < 3; ++j) memcpy(T[nt][j + 1], X[fv[j]], 3 * sizeof(double));
            ++nt;
        } else {
            double fc[3] = {0, 0, 0};
            for (int j = 0; j < 4; ++j)
                for (int a = 0; a < 3; ++a) fc[a] += 0.25 * X[fv[j]][a];
            for (int j = 0; j < 4; ++j) {
                memcpy(T[nt][0], ctr, sizeof ctr);
                memcpy(T[nt][1], X[fv[j]], 3 * sizeof(double));
                memcpy(T[nt][2], X[fv[(j + 1) % 4]], 3 * sizeof(double));
                memcpy(T[nt][3], fc, sizeof fc);
                ++nt;
            }
        }
    }
    return nt;
}

/* Volume quadrature of a cell: collapsed (Duffy) tensor Gauss-Legendre rule
 * with n points per direction on each sub-tetrahedron.  Exact for
 * polynomials of degree <= 2n-3 on each (affine) sub-tetrahedron. */
int or_cell_quad(const oracle_mesh* m, int64_t c, int n, double* xq, double* wq, int cap) {
    double T[24][4][3], gx[8], gw[8];
    int nt = cell_subtets(m, c, T);
    gauss_legendre01(n, gx, gw);
    int q = 0;
    for (int t = 0; t < nt; ++t) {
        double e1[3], e2[3], e3[3], cr[3];
        sub3(T[t][1], T[t][0], e1);
        sub3(T[t][2], T[t][0], e2);
        sub3(T[t][3], T[t][0], e3);
        cross3(e2, e3, cr);
        double det = dot3(e1, cr); /* 6 x signed volume */
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                for (int k = 0; k < n; ++k) {
                    double u = gx[i], v = gx[j], s = gx[k];
                    double a = u, b = v * (1.0 - u), cc = s * (1.0 - u) * (1.0 - v);
                    double w = gw[i] * gw[j] * gw[k] * (1.0 - u) * (1.0 - u) * (1.0 - v) * det;
                    if (q >= cap) return -1;
                    for (int d = 0; d < 3; ++d)
                        xq[3 * q + d] = T[t][0][d] + a * e1[d] + b * e2[d] + cc * e3[d];
                    wq[q] = w;
                    ++q;
                }
    }
    return q;
}

/* ------------------------------------------------------------------- faces */

typedef struct {
    int64_t key[4];
    int64_t cell;
    int lf;
} face_rec;

static int cmp_key(const int64_t* a, const int64_t* b) {
    for (int i = 0; i < 4; ++i) {
        if (a[i] < b[i]) return -1;
        if (a[i] > b[i]) return 1;
    }
    return 0;
}
static int cmp_face_rec(const void* pa, const void* pb) {
    const face_rec* a = pa;
    const face_rec* b = pb;
    int c = cmp_key(a->key, b->key);
    if (c) return c;
    if (a->cell != b->cell) return a->cell < b->cell ? -1 : 1;
    return a->lf - b->lf;
}
static void sort_key(int64_t* k, int n) {
    for (int i = 0; i < 4; ++i)
        if (i >= n) k[i] = -1;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            if (k[j] < k[i]) {
                int64_t t = k[i];
                k[i] = k[j];
                k[j] = t;
            }
}

/* Face quadrature (Sec. 2.2, eq. fv_update: points x_alpha, weights w_alpha
 * with sum w = 1).  Triangles: 3-point degree-2 rule at barycentric
 * (2/3,1/6,1/6) and permutations.  Quadrilaterals: r x r Gauss-Legendre on
 * the bilinear map, weights proportional to the map's Jacobian. */
static int face_quadrature(int nv, double V[4][3], int order, double* qp, double* qw) {
    if (nv == 3) {
        const double A = 2.0 / 3.0, B = 1.0 / 6.0;
        const double bc[3][3] = {{A, B, B}, {B, A, B}, {B, B, A}};
        for (int q = 0; q < 3; ++q) {
            for (int d = 0; d < 3; ++d)
                qp[3 * q + d] = bc[q][0] * V[0][d] + bc[q][1] * V[1][d] + bc[q][2] * V[2][d];
            qw[q] = 1.0 / 3.0;
        }
        return 3;
    }
    double gx[8], gw[8];
    int n = order;
    gauss_legendre01(n, gx, gw);
    double wsum = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double s = gx[i], t = gx[j];
            int q = i + n * j;
            double xs[3], xt[3], cr[3];
            for (int d = 0; d < 3; ++d) {
                qp[3 * q + d] = (1 - s) * (1 - t) * V[0][d] + s * (1 - t) * V[1][d] + s * t * V[2][d] +
                                (1 - s) * t * V[3][d];
                xs[d] = (1 - t) * (V[1][d] - V[0][d]) + t * (V[2][d] - V[3][d]);
                xt[d] = (1 - s) * (V[3][d] - V[0][d]) + s * (V[2][d] - V[1][d]);
            }
            cross3(xs, xt, cr);
            qw[q] = gw[i] * gw[j] * norm3(cr);
            wsum += qw[q];
        }
    for (int q = 0; q < n * n; ++q) qw[q] /= wsum;
    return n * n;
}

static int build_faces(oracle_mesh* m) {
    int64_t nc = m->n_cell, nrec = 0;
    for (int64_t c = 0; c < nc; ++c) {
        int nf = or_cell_nfaces(m->type[c]);
        if (nf < 0) return or_fail(-2, "cell %lld: unsupported type %d", (long long)c, m->type[c]);
        nrec += nf;
    }
    face_rec* rec = malloc(sizeof(face_rec) * (size_t)nrec);
    int64_t r = 0;
    for (int64_t c = 0; c < nc; ++c) {
        int type = m->type[c], nf = or_cell_nfaces(type);
        for (int lf = 0; lf < nf; ++lf) {
            int fnv;
            const int* fv = or_face_verts(type, lf, &fnv);
            for (int j = 0; j < fnv; ++j) rec[r].key[j] = m->cell_vtx[m->cell_ptr[c] + fv[j]];
            sort_key(rec[r].key, fnv);
            rec[r].cell = c;
            rec[r].lf = lf;
            ++r;
        }
    }
    qsort(rec, (size_t)nrec, sizeof(face_rec), cmp_face_rec);
    /* boundary face keys, sorted */
    face_rec* brec = malloc(sizeof(face_rec) * (size_t)(m->n_bface + 1));
    for (int64_t b = 0; b < m->n_bface; ++b) {
        int n = (int)(m->bface_ptr[b + 1] - m->bface_ptr[b]);
        for (int j = 0; j < n; ++j) brec[b].key[j] = m->bface_vtx[m->bface_ptr[b] + j];
        sort_key(brec[b].key, n);
        brec[b].cell = m->bface_tag[b];
        brec[b].lf = 0;
    }
    qsort(brec, (size_t)m->n_bface, sizeof(face_rec), cmp_face_rec);

    int64_t nf = 0;
    for (int64_t i = 0; i < nrec;) {
        int64_t j = i + 1;
        while (j < nrec && cmp_key(rec[j].key, rec[i].key) == 0) ++j;
        if (j - i > 2) {
            free(rec);
            free(brec);
            return or_fail(-2, "non-manifold face shared by %lld cells", (long long)(j - i));
        }
        ++nf;
        i = j;
    }
    m->n_face = nf;
    m->fcell = malloc(sizeof(int64_t) * 2 * nf);
    m->flf = malloc(sizeof(int32_t) * 2 * nf);
    m->fnq = malloc(sizeof(int32_t) * nf);
    m->farea = malloc(sizeof(double) * nf);
    m->fnrm = malloc(sizeof(double) * 3 * nf);
    m->fqp = calloc((size_t)nf * OR_QM * 3, sizeof(double));
    m->fqw = calloc((size_t)nf * OR_QM, sizeof(double));
    m->fshift = calloc((size_t)nf * 3, sizeof(double));
    m->fcen = malloc(sizeof(double) * 3 * nf);
    m->c2f = malloc(sizeof(int64_t) * OR_MAXF * nc);
    m->c2s = malloc(sizeof(int8_t) * OR_MAXF * nc);
    for (int64_t k = 0; k < OR_MAXF * nc; ++k) {
        m->c2f[k] = -1;
        m->c2s[k] = 0;
    }
    int64_t f = 0, nb = 0;
    for (int64_t i = 0; i < nrec;) {
        int64_t j = i + 1;
        while (j < nrec && cmp_key(rec[j].key, rec[i].key) == 0) ++j;
        /* owner = lower cell id (records are sorted by cell within a key) */
        m->fcell[2 * f] = rec[i].cell;
        m->flf[2 * f] = rec[i].lf;
        m->c2f[OR_MAXF * rec[i].cell + rec[i].lf] = f;
        m->c2s[OR_MAXF * rec[i].cell + rec[i].lf] = 0;
        if (j - i == 2) {
            if (rec[i + 1].cell == rec[i].cell) {
                free(rec);
                free(brec);
                return or_fail(-2, "cell %lld meets itself through a face", (long long)rec[i].cell);
            }
            m->fcell[2 * f + 1] = rec[i + 1].cell;
            m->flf[2 * f + 1] = rec[i + 1].lf;
            m->c2f[OR_MAXF * rec[i + 1].cell + rec[i + 1].lf] = f;
            m->c2s[OR_MAXF * rec[i + 1].cell + rec[i + 1].lf] = 1;
        } else {
            /* boundary: find tag by binary search */
            int64_t lo = 0, hi = m->n_bface - 1, tag = -1;
            while (lo <= hi) {
                int64_t mid = (lo + hi) / 2;
                int cm = cmp_key(brec[mid].key, rec[i].key);
                if (cm == 0) {
                    tag = brec[mid].cell;
                    break;
                }
                if (cm < 0)
                    lo = mid + 1;
                else
                    hi = mid - 1;
            }
            if (tag < 1 || tag > 7) {
                free(rec);
                free(brec);
                return or_fail(-2, "unmatched face of cell %lld (no neighbour, no boundary tag)",
                               (long long)rec[i].cell);
            }
            m->fcell[2 * f + 1] = -1 - tag;
            m->flf[2 * f + 1] = -1;
            ++nb;
        }
        ++f;
        i = j;
    }
    m->n_bnd = nb;
    free(rec);
    free(brec);

    /* Face geometry in the owner's frame. */
    for (f = 0; f < nf; ++f) {
        int64_t cL = m->fcell[2 * f];
        int type = m->type[cL], fnv;
        const int* fv = or_face_verts(type, m->flf[2 * f], &fnv);
        double X[8][3], V[4][3], vec[3];
        or_cell_coords(m, cL, X);
        for (int j = 0; j < fnv; ++j) memcpy(V[j], X[fv[j]], sizeof V[j]);
        if (fnv == 3) {
            double e1[3], e2[3];
            sub3(V[1], V[0], e1);
            sub3(V[2], V[0], e2);
            cross3(e1, e2, vec);
        } else {
            double d1[3], d2[3];
            sub3(V[2], V[0], d1);
            sub3(V[3], V[1], d2);
            cross3(d1, d2, vec);
        }
        for (int a = 0; a < 3; ++a) vec[a] *= 0.5;
        double ar = norm3(vec);
        m->farea[f] = ar;
        for (int a = 0; a < 3; ++a) m->fnrm[3 * f + a] = vec[a] / ar;
        for (int a = 0; a < 3; ++a) {
            double s = 0;
            for (int j = 0; j < fnv; ++j) s += V[j][a];
            m->fcen[3 * f + a] = s / fnv;
        }
        m->fnq[f] = face_quadrature(fnv, V, m->order, m->fqp + (size_t)f * OR_QM * 3, m->fqw + (size_t)f * OR_QM);
        int64_t cR = m->fcell[2 * f + 1];
        if (cR >= 0) {
            /* shift such that (neighbour frame) = (owner frame) - shift */
            double XR[8][3];
            or_cell_coords(m, cR, XR);
            int64_t gv = m->cell_vtx[m->cell_ptr[cL] + fv[0]];
            int kR = -1;
            for (int k = 0; k < m->cell_ptr[cR + 1] - m->cell_ptr[cR]; ++k)
                if (m->cell_vtx[m->cell_ptr[cR] + k] == gv) kR = k;
            for (int a = 0; a < 3; ++a) {
                double d = V[0][a] - XR[kR][a];
                m->fshift[3 * f + a] = m->period[a] > 0.0 ? m->period[a] * nearbyint(d / m->period[a]) : 0.0;
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------------- cell geometry */

static void build_cell_geometry(oracle_mesh* m) {
    int64_t nc = m->n_cell;
    m->vol = malloc(sizeof(double) * nc);
    m->cen = malloc(sizeof(double) * 3 * nc);
    m->hbasis = malloc(sizeof(double) * nc);
    m->hdt = malloc(sizeof(double) * nc);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        double xq[OR_VQ * 3], wq[OR_VQ];
        int n = or_cell_quad(m, c, 2, xq, wq, OR_VQ);
        double V = 0, C[3] = {0, 0, 0};
        for (int q = 0; q < n; ++q) {
            V += wq[q];
            for (int a = 0; a < 3; ++a) C[a] += wq[q] * xq[3 * q + a];
        }
        for (int a = 0; a < 3; ++a) C[a] /= V;
        m->vol[c] = V;
        memcpy(m->cen + 3 * c, C, sizeof C);
        double X[8][3], h = 0;
        int nv = or_cell_coords(m, c, X);
        for (int k = 0; k < nv; ++k) {
            double d[3];
            sub3(X[k], C, d);
            double r = norm3(d);
            if (r > h) h = r;
        }
        m->hbasis[c] = h;
        double S = 0;
        for (int lf = 0; lf < or_cell_nfaces(m->type[c]); ++lf) S += m->farea[m->c2f[OR_MAXF * c + lf]];
        m->hdt[c] = 6.0 * V / S;
    }
}

/* ----------------------------------------------------------------- stencils */

typedef struct {
    double dist;
    int64_t id;
    double d[3];
} cand;

static int cmp_cand(const void* pa, const void* pb) {
    const cand* a = pa;
    const cand* b = pb;
    if (a->dist < b->dist) return -1;
    if (a->dist > b->dist) return 1;
    return a->id < b->id ? -1 : (a->id > b->id);
}

/* Stencil selection (Sec. 2.2: compact central and directional stencils; the
 * paper cites the selection algorithm without stating it).  Reading:
 *  - candidate pool: cells within L vertex-neighbour layers, L the smallest
 *    value >= 2 with at least 2*Mc candidates, capped at max_layers;
 *  - central stencil: the Mc = round(f K(r,3)) nearest centroids, f the
 *    stencil factor (2 by default: twice the basis size; periodic minimum
 *    image), extended by every candidate within (1 + 1e-9) of the Mc-th
 *    distance ("shell closure", so ties never split);
 *  - one directional stencil per face: candidates whose centroid lies in the
 *    closed cone from the cell centroid through the face's vertices (1e-9
 *    relative tolerance), the 8 nearest with shell closure; fewer than 4
 *    candidates drops the stencil. */
static int build_stencil(const oracle_mesh* m, int64_t c, const int64_t* v2c_ptr, const int64_t* v2c,
                         char* mark, int64_t* list, cand* pool, oracle_stencil_t* st) {
    int K = m->K, Mc = (int)lround(m->stencil_factor * (K + 1));
    int64_t npool = 0;
    /* BFS over vertex adjacency */
    int64_t head = 0;
    list[npool++] = c;
    mark[c] = 1;
    int64_t layer_end = 1;
    int L = 0;
    while (1) {
        int64_t stop = layer_end;
        for (; head < stop; ++head) {
            int64_t cc = list[head];
            for (int64_t p = m->cell_ptr[cc]; p < m->cell_ptr[cc + 1]; ++p) {
                int64_t v = m->cell_vtx[p];
                for (int64_t q = v2c_ptr[v]; q < v2c_ptr[v + 1]; ++q) {
                    int64_t nb = v2c[q];
                    if (!mark[nb]) {
                        mark[nb] = 1;
                        list[npool++] = nb;
                    }
                }
            }
        }
        layer_end = npool;
        ++L;
        if ((L >= 2 && npool - 1 >= 2 * Mc) || L >= m->max_layers || head == npool) break;
    }
    for (int64_t k = 0; k < npool; ++k) mark[list[k]] = 0;
    int64_t ncand = 0;
    for (int64_t k = 1; k < npool; ++k) {
        int64_t id = list[k];
        cand* p = &pool[ncand++];
        p->id = id;
        sub3(m->cen + 3 * id, m->cen + 3 * c, p->d);
        min_image(m, p->d);
        p->dist = norm3(p->d);
    }
    qsort(pool, (size_t)ncand, sizeof(cand), cmp_cand);
    /* central */
    int n = ncand < Mc ? (int)ncand : Mc;
    if (n < K) return or_fail(-3, "cell %lld: only %d stencil candidates for %d unknowns", (long long)c, n, K);
    double dlim = pool[n - 1].dist * (1.0 + 1e-9);
    while (n < ncand && pool[n].dist <= dlim) ++n;
    if (n > OR_MAXM) return or_fail(-2, "cell %lld: central stencil of %d exceeds %d", (long long)c, n, OR_MAXM);
    st->ncen = n;
    st->navail = ncand < OR_MAXM ? (int)ncand : OR_MAXM;
    for (int k = 0; k < st->navail; ++k) {
        st->cen[k] = pool[k].id;
        st->cdist[k] = pool[k].dist;
    }
    /* directional */
    double X[8][3];
    or_cell_coords(m, c, X);
    const double* ci = m->cen + 3 * c;
    int type = m->type[c], nf = or_cell_nfaces(type);
    st->ndir = 0;
    for (int lf = 0; lf < nf; ++lf) {
        int fnv;
        const int* fv = or_face_verts(type, lf, &fnv);
        double v[4][3], nrm[4][3], fc[3] = {0, 0, 0};
        for (int j = 0; j < fnv; ++j) {
            sub3(X[fv[j]], ci, v[j]);
            for (int a = 0; a < 3; ++a) fc[a] += v[j][a] / fnv;
        }
        for (int j = 0; j < fnv; ++j) {
            cross3(v[j], v[(j + 1) % fnv], nrm[j]);
            if (dot3(nrm[j], fc) < 0)
                for (int a = 0; a < 3; ++a) nrm[j][a] = -nrm[j][a];
        }
        /* 2 K(d,3) nearest (8 for linear, 20 for quadratic polynomials),
         * at least K(d,3) (4 / 10) or the sector is dropped */
        const int target = 2 * (m->kd + 1), least = m->kd + 1;
        int cnt = 0, s = st->ndir;
        int64_t ids[OR_MAXMD];
        double lim = -1.0;
        for (int64_t k = 0; k < ncand; ++k) {
            const double* d = pool[k].d;
            int inside = 1;
            for (int j = 0; j < fnv && inside; ++j)
                if (dot3(d, nrm[j]) < -1e-9 * pool[k].dist * norm3(nrm[j])) inside = 0;
            if (!inside) continue;
            if (cnt >= target && pool[k].dist > lim) break;
            if (cnt >= OR_MAXMD) return or_fail(-2, "cell %lld: directional stencil overflow", (long long)c);
            ids[cnt] = pool[k].id;
            ++cnt;
            if (cnt == target) lim = pool[k].dist * (1.0 + 1e-9);
        }
        if (cnt < least) {
            st->ndropped++;
            continue;
        }
        st->dface[s] = lf;
        st->nd[s] = cnt;
        for (int k = 0; k < cnt; ++k) st->dir[s][k] = ids[k];
        st->ndir++;
    }
    return 0;
}

/* ------------------------------------------------------- least squares (QR) */

/* Least-squares operator B = A^+ diag(w) of an (n x k) system, A row-major,
 * by Householder QR of the column-equilibrated matrix (Sec. 2.2: "pseudo-
 * inverse QR-based operators precomputed").  Returns the smallest ratio
 * |R_jj| / |R_11| through *rcond.  B is (k x n) row-major. */
int or_lsq_operator(int n, int k, const double* A, const double* w, double* B, double* rcond) {
    double Q[OR_MAXM * OR_MAXM], R[OR_MAXM * OR_MAXK], colscale[OR_MAXK];
    for (int j = 0; j < k; ++j) {
        double s = 0;
        for (int i = 0; i < n; ++i) s += A[i * k + j] * A[i * k + j];
        colscale[j] = s > 0 ? 1.0 / sqrt(s) : 1.0;
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < k; ++j) R[i * k + j] = A[i * k + j] * colscale[j];
    /* Q^T accumulated as an n x n matrix, starting from the identity */
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Q[i * n + j] = (i == j);
    for (int j = 0; j < k; ++j) {
        double alpha = 0;
        for (int i = j; i < n; ++i) alpha += R[i * k + j] * R[i * k + j];
        alpha = sqrt(alpha);
        if (R[j * k + j] > 0) alpha = -alpha;
        double v[OR_MAXM];
        for (int i = 0; i < n; ++i) v[i] = 0;
        for (int i = j; i < n; ++i) v[i] = R[i * k + j];
        v[j] -= alpha;
        double vv = 0;
        for (int i = j; i < n; ++i) vv += v[i] * v[i];
        if (vv == 0) continue;
        for (int c = 0; c < k; ++c) {
            double s = 0;
            for (int i = j; i < n; ++i) s += v[i] * R[i * k + c];
            s = 2 * s / vv;
            for (int i = j; i < n; ++i) R[i * k + c] -= s * v[i];
        }
        for (int c = 0; c < n; ++c) {
            double s = 0;
            for (int i = j; i < n; ++i) s += v[i] * Q[i * n + c];
            s = 2 * s / vv;
            for (int i = j; i < n; ++i) Q[i * n + c] -= s * v[i];
        }
    }
    double r11 = fabs(R[0]), rmin = r11;
    for (int j = 0; j < k; ++j)
        if (fabs(R[j * k + j]) < rmin) rmin = fabs(R[j * k + j]);
    *rcond = r11 > 0 ? rmin / r11 : 0;
    if (rmin == 0) return -1;
    /* B = D R^{-1} (Q^T)[0:k,:] diag(w) */
    for (int c = 0; c < n; ++c) {
        double y[OR_MAXK];
        for (int j = k - 1; j >= 0; --j) {
            double s = Q[j * n + c];
            for (int l = j + 1; l < k; ++l) s -= R[j * k + l] * y[l];
            y[j] = s / R[j * k + j];
        }
        for (int j = 0; j < k; ++j) B[j * n + c] = colscale[j] * y[j] * w[c];
    }
    return 0;
}

/* -------------------------------------------------------- cell operators */

/* Basis (Sec. 2.2, eq. lsq_poly): phi_k(x) = m_k((x - c_i)/h_i) - <m_k>_i,
 * m_k the graded-lex monomials of degree 1..r, zero mean over cell i. */
static void eval_basis(const oracle_mesh* m, int64_t c, const double* x, const double* mean, double* phi) {
    const double* ci = m->cen + 3 * c;
    double h = m->hbasis[c];
    double xi[3] = {(x[0] - ci[0]) / h, (x[1] - ci[1]) / h, (x[2] - ci[2]) / h};
    for (int k = 0; k < m->K; ++k)
        phi[k] = ipow(xi[0], m->expo[k][0]) * ipow(xi[1], m->expo[k][1]) * ipow(xi[2], m->expo[k][2]) -
                 (mean ? mean[k] : 0.0);
}

static int build_operators(oracle_mesh* m, int64_t c, oracle_stencil_t* st, oracle_ops_t* op) {
    int K = m->K, r = m->order;
    size_t nval = (size_t)K * OR_MAXM + (size_t)K * K + (size_t)OR_MAXF * OR_QM * K;
    for (int s = 0; s < st->ndir; ++s) nval += (size_t)m->kd * st->nd[s];
    double* blk = calloc(nval, sizeof(double));
    op->Bc = blk;
    blk += (size_t)K * OR_MAXM;
    op->O = blk;
    blk += (size_t)K * K;
    op->Phi = blk;
    blk += (size_t)OR_MAXF * OR_QM * K;
    for (int s = 0; s < st->ndir; ++s) {
        op->Bd[s] = blk;
        blk += (size_t)m->kd * st->nd[s];
    }
    int nvq = r + 1; /* exact for degree <= 2r-1 on every sub-tetrahedron: covers
                        the means (degree r), A (degree r) and O (degree 2r-2) */
    double xq[OR_VQ * 3], wq[OR_VQ], phi[OR_MAXK];
    int n = or_cell_quad(m, c, nvq, xq, wq, OR_VQ);
    double Vi = m->vol[c];
    /* means of the monomials over the cell */
    double mean[OR_MAXK];
    for (int k = 0; k < K; ++k) mean[k] = 0;
    for (int q = 0; q < n; ++q) {
        eval_basis(m, c, xq + 3 * q, NULL, phi);
        for (int k = 0; k < K; ++k) mean[k] += wq[q] * phi[k];
    }
    for (int k = 0; k < K; ++k) mean[k] /= Vi;
    memcpy(op->mean, mean, sizeof(double) * K);

    /* Least-squares matrix of a stencil (Sec. 2.2, eq. lsq_system):
     * A_mk = integral over cell m (periodic image nearest cell c) of phi_k,
     * right-hand side |V_m| (U_m - U_c), so B = A^+ diag(|V_m|).
     * A central stencil whose QR shows |R_jj|/|R_11| < 1e-6 is extended by
     * the next distance shell until it is well conditioned: a one-sided
     * stencil at a boundary can miss a whole direction, and a stencil of thin
     * boundary-layer prisms spans the quadratic terms only barely (condition
     * numbers near 1e7, where two correct solves agree to about 1e-9). */
    double A[OR_MAXM * OR_MAXK], w[OR_MAXM], rc;
    for (int s = -1; s < st->ndir; ++s) {
    retry:;
        int ns = s < 0 ? st->ncen : st->nd[s];
        int kk = s < 0 ? K : m->kd;
        for (int j = 0; j < ns; ++j) {
            int64_t id = s < 0 ? st->cen[j] : st->dir[s][j];
            /* shift of cell id's own frame to its image next to cell c */
            double dm[3], shift[3];
            sub3(m->cen + 3 * id, m->cen + 3 * c, dm);
            min_image(m, dm);
            for (int a = 0; a < 3; ++a) shift[a] = m->cen[3 * c + a] + dm[a] - m->cen[3 * id + a];
            double xm[OR_VQ * 3], wm[OR_VQ];
            int nm = or_cell_quad(m, id, nvq, xm, wm, OR_VQ);
            double row[OR_MAXK];
            for (int k = 0; k < K; ++k) row[k] = 0;
            for (int q = 0; q < nm; ++q) {
                double x[3] = {xm[3 * q] + shift[0], xm[3 * q + 1] + shift[1], xm[3 * q + 2] + shift[2]};
                eval_basis(m, c, x, mean, phi);
                for (int k = 0; k < kk; ++k) row[k] += wm[q] * phi[k];
            }
            for (int k = 0; k < kk; ++k) A[j * kk + k] = row[k];
            w[j] = m->vol[id];
        }
        double* B = s < 0 ? op->Bc : op->Bd[s];
        int rcq = or_lsq_operator(ns, kk, A, w, B, &rc);
        /* A directional stencil whose members cannot fix a linear
         * polynomial (all in one plane through the cell centroid, as on thin
         * boundary-layer cells: a column of A vanishes up to rounding, which
         * the unit-norm column scaling of the solve would hide) is dropped
         * like one with too few candidates; the later stencils (and their
         * operator blocks) move down one slot. */
        double cmin = INFINITY, cmax = 0;
        if (s >= 0)
            for (int k = 0; k < kk; ++k) {
                double cn = 0;
                for (int j = 0; j < ns; ++j) cn += A[j * kk + k] * A[j * kk + k];
                cmin = fmin(cmin, sqrt(cn));
                cmax = fmax(cmax, sqrt(cn));
            }
        if (s >= 0 && (rcq != 0 || rc < 1e-9 || cmin < 1e-8 * cmax)) {
            for (int t = s; t + 1 < st->ndir; ++t) {
                st->nd[t] = st->nd[t + 1];
                st->dface[t] = st->dface[t + 1];
                memcpy(st->dir[t], st->dir[t + 1], sizeof(st->dir[t]));
                op->Bd[t] = op->Bd[t + 1];
            }
            st->ndir--;
            st->ndropped++;
            if (s < st->ndir) goto retry;
            break;
        }
        if (s < 0 && (rcq != 0 || rc < 1e-6)) {
            if (st->ncen >= st->navail)
                return or_fail(-3, "cell %lld: central stencil rank deficient (rcond %g)", (long long)c, rc);
            double lim = st->cdist[st->ncen] * (1.0 + 1e-9);
            int n2 = st->ncen;
            while (n2 < st->navail && st->cdist[n2] <= lim) ++n2;
            if (n2 == OR_MAXM && st->navail > n2 - 1 && st->cdist[n2 - 1] > lim)
                return or_fail(-2, "cell %lld: central stencil cap reached", (long long)c);
            st->ncen = n2;
            goto retry;
        }
    }

    /* Oscillation matrix (reading of the smoothness indicator SI_s of
     * eq. cwenoz_weights, which the paper names without defining):
     * O_kl = sum_{1<=|b|<=r} |V|^{2|b|/3-1} integral_V D^b phi_k D^b phi_l,
     * derivatives in physical coordinates, each multi-index b once. */
    for (int k = 0; k < K * K; ++k) op->O[k] = 0;
    int nb = 0, beta[OR_MAXK][3];
    monomial_exponents(r, beta);
    nb = K;
    /* D^b phi_k vanishes identically unless every exponent of phi_k reaches
     * b's: only those k enter the sum for b (the skipped terms are exact
     * zeros, so the sum is unchanged) */
    int nzk[OR_MAXK][OR_MAXK], nnz[OR_MAXK];
    for (int b = 0; b < nb; ++b) {
        nnz[b] = 0;
        for (int k = 0; k < K; ++k)
            if (m->expo[k][0] >= beta[b][0] && m->expo[k][1] >= beta[b][1] && m->expo[k][2] >= beta[b][2])
                nzk[b][nnz[b]++] = k;
    }
    for (int q = 0; q < n; ++q) {
        const double* ci = m->cen + 3 * c;
        double h = m->hbasis[c];
        double xi[3] = {(xq[3 * q] - ci[0]) / h, (xq[3 * q + 1] - ci[1]) / h, (xq[3 * q + 2] - ci[2]) / h};
        for (int b = 0; b < nb; ++b) {
            int ord = beta[b][0] + beta[b][1] + beta[b][2];
            double scale = pow(Vi, 2.0 * ord / 3.0 - 1.0) * ipow(1.0 / h, 2 * ord);
            double D[OR_MAXK];
            for (int i = 0; i < nnz[b]; ++i) {
                int k = nzk[b][i];
                double v = 1.0;
                for (int a = 0; a < 3; ++a) {
                    int e = m->expo[k][a], bb = beta[b][a];
                    double fac = 1.0;
                    for (int t = 0; t < bb; ++t) fac *= (double)(e - t);
                    v *= fac * ipow(xi[a], e - bb);
                }
                D[k] = v;
            }
            for (int i = 0; i < nnz[b]; ++i)
                for (int j = 0; j < nnz[b]; ++j) {
                    int k = nzk[b][i], l = nzk[b][j];
                    op->O[k * K + l] += wq[q] * scale * D[k] * D[l];
                }
        }
    }

    /* Basis values at the cell's own face quadrature points; the neighbour
     * side evaluates at the owner's points moved into its frame. */
    int type = m->type[c];
    for (int lf = 0; lf < or_cell_nfaces(type); ++lf) {
        int64_t f = m->c2f[OR_MAXF * c + lf];
        int side = m->c2s[OR_MAXF * c + lf];
        for (int q = 0; q < m->fnq[f]; ++q) {
            double x[3];
            for (int a = 0; a < 3; ++a)
                x[a] = m->fqp[((size_t)f * OR_QM + q) * 3 + a] - (side ? m->fshift[3 * f + a] : 0.0);
            eval_basis(m, c, x, mean, op->Phi + (size_t)(lf * OR_QM + q) * K);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------- build */

int oracle_build(const oracle_mesh_in* in, const oracle_opts* opt, const uint8_t* need, int n_threads,
                 oracle_mesh** out) {
    (void)n_threads;
    if (!in || !opt || !out) return or_fail(-1, "null argument");
    if (opt->order < 1 || opt->order > 4) return or_fail(-1, "order %d not supported", opt->order);
    if (opt->tri_qp != 3) return or_fail(-1, "only the 3-point triangle rule is implemented");
    oracle_mesh* m = calloc(1, sizeof(oracle_mesh));
    m->n_vert = in->n_vert;
    m->n_cell = in->n_cell;
    m->xyz = in->xyz;
    m->type = in->type;
    m->cell_ptr = in->cell_ptr;
    m->cell_vtx = in->cell_vtx;
    memcpy(m->period, in->period, sizeof m->period);
    m->n_bface = in->n_bface;
    m->bface_ptr = in->bface_ptr;
    m->bface_vtx = in->bface_vtx;
    m->bface_tag = in->bface_tag;
    m->order = opt->order;
    m->K = or_K(opt->order) - 1;
    /* directional polynomials: linear for the third- and fourth-order
     * schemes, quadratic from the fifth order on (Sec. 2.2) */
    m->kd = opt->order >= 4 ? or_K(2) - 1 : or_K(1) - 1;
    if (opt->order >= 4)
        for (int64_t c = 0; c < in->n_cell; ++c)
            if (in->type[c] != 8) {
                free(m);
                return or_fail(-1, "order %d is built for hexahedral meshes only (the 3-point triangle rule is "
                                   "exact to degree 2)", opt->order);
            }
    m->lambda_c = opt->lambda_c;
    m->eps = opt->eps;
    m->max_layers = opt->max_layers;
    m->stencil_factor = opt->stencil_factor > 0 ? opt->stencil_factor : 2.0;
    monomial_exponents(m->order, m->expo);
    int rc = build_faces(m);
    if (rc) {
        oracle_free(m);
        return rc;
    }
    build_cell_geometry(m);
    for (int64_t c = 0; c < m->n_cell; ++c)
        if (m->vol[c] <= 0) {
            oracle_free(m);
            return or_fail(-2, "cell %lld has non-positive volume", (long long)c);
        }

    /* vertex -> cells */
    int64_t nv = m->n_vert, nc = m->n_cell;
    int64_t* v2c_ptr = calloc((size_t)nv + 1, sizeof(int64_t));
    for (int64_t p = 0; p < m->cell_ptr[nc]; ++p) v2c_ptr[m->cell_vtx[p] + 1]++;
    for (int64_t v = 0; v < nv; ++v) v2c_ptr[v + 1] += v2c_ptr[v];
    int64_t* v2c = malloc(sizeof(int64_t) * (size_t)m->cell_ptr[nc]);
    int64_t* fill = calloc((size_t)nv, sizeof(int64_t));
    for (int64_t c = 0; c < nc; ++c)
        for (int64_t p = m->cell_ptr[c]; p < m->cell_ptr[c + 1]; ++p) {
            int64_t v = m->cell_vtx[p];
            v2c[v2c_ptr[v] + fill[v]++] = c;
        }
    free(fill);

    m->need = malloc(nc);
    for (int64_t c = 0; c < nc; ++c) m->need[c] = need ? (need[c] != 0) : 1;
    m->st = calloc((size_t)nc, sizeof(oracle_stencil_t*));
    m->op = calloc((size_t)nc, sizeof(oracle_ops_t*));
    int err = 0;
    char errmsg[512] = {0};
#pragma omp parallel
    {
        char* mark = calloc((size_t)nc, 1);
        int64_t* list = malloc(sizeof(int64_t) * (size_t)nc);
        cand* pool = malloc(sizeof(cand) * (size_t)nc);
#pragma omp for schedule(dynamic, 64)
        for (int64_t c = 0; c < nc; ++c) {
            if (!m->need[c] || err) continue;
            oracle_stencil_t* st = calloc(1, sizeof(oracle_stencil_t));
            oracle_ops_t* op = calloc(1, sizeof(oracle_ops_t));
            int e = build_stencil(m, c, v2c_ptr, v2c, mark, list, pool, st);
            if (!e) e = build_operators(m, c, st, op);
            m->st[c] = st;
            m->op[c] = op;
            if (e) {
#pragma omp critical
                {
                    if (!err) {
                        err = e;
                        strncpy(errmsg, g_err, sizeof errmsg - 1);
                    }
                }
            }
        }
        free(mark);
        free(list);
        free(pool);
    }
    free(v2c_ptr);
    free(v2c);
    if (err) {
        oracle_free(m);
        strncpy(g_err, errmsg, sizeof g_err - 1);
        return err;
    }
    *out = m;
    return 0;
}

void oracle_free(oracle_mesh* m) {
    if (!m) return;
    if (m->st)
        for (int64_t c = 0; c < m->n_cell; ++c) {
            free(m->st[c]);
            if (m->op[c]) free(m->op[c]->Bc);
            free(m->op[c]);
        }
    free(m->st);
    free(m->op);
    free(m->need);
    free(m->fcell);
    free(m->flf);
    free(m->fnq);
    free(m->farea);
    free(m->fnrm);
    free(m->fqp);
    free(m->fqw);
    free(m->fshift);
    free(m->fcen);
    free(m->c2f);
    free(m->c2s);
    free(m->vol);
    free(m->cen);
    free(m->hbasis);
    free(m->hdt);
    free(m);
}

/* ---------------------------------------------------------------- getters */

int oracle_info(const oracle_mesh* m, int64_t* info) {
    int64_t maxc = 0, minc = 1 << 30, maxd = 0, nq = 0, nfc = 0, ndrop = 0;
    for (int64_t f = 0; f < m->n_face; ++f)
        if (m->fnq[f] > nq) nq = m->fnq[f];
    for (int64_t c = 0; c < m->n_cell; ++c) {
        int nf = or_cell_nfaces(m->type[c]);
        if (nf > nfc) nfc = nf;
        if (!m->st[c]) continue;
        if (m->st[c]->ncen > maxc) maxc = m->st[c]->ncen;
        if (m->st[c]->ncen < minc) minc = m->st[c]->ncen;
        for (int s = 0; s < m->st[c]->ndir; ++s)
            if (m->st[c]->nd[s] > maxd) maxd = m->st[c]->nd[s];
        ndrop += m->st[c]->ndropped;
    }
    info[0] = m->n_cell;
    info[1] = m->n_face;
    info[2] = m->K;
    info[3] = nq;
    info[4] = nfc;
    info[5] = maxc;
    info[6] = maxd;
    info[7] = minc;
    info[8] = m->n_bnd;
    info[9] = ndrop;
    info[10] = m->kd;
    return 0;
}

int oracle_cell_faces(const oracle_mesh* m, int64_t* c2f, int8_t* side) {
    memcpy(c2f, m->c2f, sizeof(int64_t) * OR_MAXF * m->n_cell);
    memcpy(side, m->c2s, OR_MAXF * m->n_cell);
    return 0;
}

int oracle_face_data(const oracle_mesh* m, int64_t* cells, int32_t* nq, double* area, double* nrm, double* qp,
                     double* qw, double* shift) {
    int64_t nf = m->n_face;
    if (cells) memcpy(cells, m->fcell, sizeof(int64_t) * 2 * nf);
    if (nq) memcpy(nq, m->fnq, sizeof(int32_t) * nf);
    if (area) memcpy(area, m->farea, sizeof(double) * nf);
    if (nrm) memcpy(nrm, m->fnrm, sizeof(double) * 3 * nf);
    if (qp) memcpy(qp, m->fqp, sizeof(double) * 3 * OR_QM * nf);
    if (qw) memcpy(qw, m->fqw, sizeof(double) * OR_QM * nf);
    if (shift) memcpy(shift, m->fshift, sizeof(double) * 3 * nf);
    return 0;
}

int oracle_cell_data(const oracle_mesh* m, double* vol, double* cen, double* hbasis) {
    if (vol) memcpy(vol, m->vol, sizeof(double) * m->n_cell);
    if (cen) memcpy(cen, m->cen, sizeof(double) * 3 * m->n_cell);
    if (hbasis) memcpy(hbasis, m->hbasis, sizeof(double) * m->n_cell);
    return 0;
}

int oracle_stencil(const oracle_mesh* m, int64_t cell, int64_t* central, int32_t* ncen, int64_t* dir, int32_t* ndir,
                   int32_t* dface) {
    const oracle_stencil_t* st = m->st[cell];
    if (!st) return or_fail(-1, "cell %lld not built", (long long)cell);
    *ncen = st->ncen;
    for (int k = 0; k < st->ncen; ++k) central[k] = st->cen[k];
    for (int s = 0; s < st->ndir; ++s) {
        ndir[s] = st->nd[s];
        dface[s] = st->dface[s];
        for (int k = 0; k < st->nd[s]; ++k) dir[s * OR_MAXMD + k] = st->dir[s][k];
    }
    return st->ndir;
}

int oracle_operators(const oracle_mesh* m, int64_t cell, double* Bc, double* Bd, double* O, double* Phi,
                     double* mean) {
    const oracle_stencil_t* st = m->st[cell];
    const oracle_ops_t* op = m->op[cell];
    if (!st) return or_fail(-1, "cell %lld not built", (long long)cell);
    int K = m->K;
    if (Bc) memcpy(Bc, op->Bc, sizeof(double) * K * st->ncen);
    if (Bd)
        for (int s = 0; s < st->ndir; ++s)
            memcpy(Bd + (size_t)s * m->kd * OR_MAXMD, op->Bd[s], sizeof(double) * m->kd * st->nd[s]);
    if (O) memcpy(O, op->O, sizeof(double) * K * K);
    if (Phi) memcpy(Phi, op->Phi, sizeof(double) * OR_MAXF * OR_QM * K);
    if (mean) memcpy(mean, op->mean, sizeof(double) * K);
    return 0;
}

int oracle_cell_quadrature(const oracle_mesh* m, int64_t cell, double* x, double* w, int cap) {
    return or_cell_quad(m, cell, m->order + 1, x, w, cap);
}
