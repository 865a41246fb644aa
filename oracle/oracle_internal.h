/* FP64 oracle internals (test infrastructure only). */
#ifndef UCNS_ORACLE_INTERNAL_H
#define UCNS_ORACLE_INTERNAL_H
#include "oracle.h"

#define OR_MAXF 6    /* faces per cell */
#define OR_QM 16     /* quadrature points per face (4x4 at r = 4) */
#define OR_MAXK 34   /* unknowns at r = 4 */
#define OR_MAXKD 9   /* unknowns of a directional polynomial (quadratic) */
#define OR_MAXM 128  /* central stencil size cap */
#define OR_MAXMD 32  /* directional stencil size cap */
#define OR_VQ 3000   /* volume quadrature points per cell (24 sub-tets x 5^3) */

typedef struct {
    int ncen, navail;           /* central size; sorted candidates kept */
    int64_t cen[OR_MAXM];       /* the first navail candidates by (distance, id) */
    double cdist[OR_MAXM];
    int ndir, ndropped;
    int nd[OR_MAXF];
    int dface[OR_MAXF];
    int64_t dir[OR_MAXF][OR_MAXMD];
} oracle_stencil_t;

typedef struct {
    double mean[OR_MAXK];
    double* Bc;          /* [K][ncen] */
    double* Bd[OR_MAXF]; /* [kd][nd[s]] */
    double* O;           /* [K][K] */
    double* Phi;         /* [OR_MAXF * OR_QM][K] */
} oracle_ops_t;

struct oracle_mesh {
    int64_t n_vert, n_cell, n_face, n_bface, n_bnd;
    const double* xyz;
    const uint8_t* type;
    const int64_t* cell_ptr;
    const int64_t* cell_vtx;
    double period[3];
    const int64_t* bface_ptr;
    const int64_t* bface_vtx;
    const int32_t* bface_tag;
    int order, K, max_layers;
    int kd;          /* unknowns of the directional polynomials: 3 (linear, r <= 3) or 9 (quadratic, r >= 4) */
    double stencil_factor;
    double lambda_c, eps;
    int expo[OR_MAXK][3];
    /* faces */
    int64_t* fcell;  /* [nf][2]; side 1 = -1 - tag on boundary */
    int32_t* flf;    /* [nf][2] local face index */
    int32_t* fnq;
    double *farea, *fnrm, *fqp, *fqw, *fshift, *fcen;
    int64_t* c2f;    /* [nc][OR_MAXF] */
    int8_t* c2s;
    /* cells */
    double *vol, *cen, *hbasis, *hdt;
    uint8_t* need;
    oracle_stencil_t** st;
    oracle_ops_t** op;
};

int or_fail(int code, const char* fmt, ...);
int or_cell_nfaces(int type);
const int* or_face_verts(int type, int lf, int* nv);
int or_K(int r);
int or_cell_coords(const oracle_mesh* m, int64_t c, double X[8][3]);
int or_cell_quad(const oracle_mesh* m, int64_t c, int n, double* xq, double* wq, int cap);
int or_lsq_operator(int n, int k, const double* A, const double* w, double* B, double* rcond);

#endif
