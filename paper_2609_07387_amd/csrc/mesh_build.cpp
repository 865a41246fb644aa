// Host mesh build of libucns: faces, geometry, quadrature, basis, stencils and
// least-squares reconstruction operators, all in FP64, multithreaded.
//
// Method: Sec. 2.2 of the UCNS3D v4 paper (eqs. lsq_poly, lsq_system,
// cwenoz_weights, fv_update).  Volume integrals use cell moments about the
// centroid and binomial re-centring; the least-squares pseudo-inverse uses
// column-equilibrated modified Gram-Schmidt QR with re-orthogonalisation.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "ucns_internal.hpp"

namespace ucns {

// --------------------------------------------------------------- topology
// Local faces with outward right-hand orientation (tet/hex: VTK numbering).
namespace {
const int kTetFaces[4][4] = {{1, 2, 3, -1}, {0, 3, 2, -1}, {0, 1, 3, -1}, {0, 2, 1, -1}};
const int kPyrFaces[5][4] = {{0, 3, 2, 1}, {0, 1, 4, -1}, {1, 2, 4, -1}, {2, 3, 4, -1}, {3, 0, 4, -1}};
const int kPrismFaces[5][4] = {{0, 2, 1, -1}, {3, 4, 5, -1}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}};
const int kHexFaces[6][4] = {{0, 4, 7, 3}, {1, 2, 6, 5}, {0, 1, 5, 4}, {3, 7, 6, 2}, {0, 3, 2, 1}, {4, 5, 6, 7}};

using Vec3 = std::array<double, 3>;
inline Vec3 operator-(const Vec3& a, const Vec3& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
inline Vec3 operator+(const Vec3& a, const Vec3& b) { return {a[0] + b[0], a[1] + b[1], a[2] + b[2]}; }
inline Vec3 operator*(double s, const Vec3& a) { return {s * a[0], s * a[1], s * a[2]}; }
inline double dot(const Vec3& a, const Vec3& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline Vec3 cross(const Vec3& a, const Vec3& b) {
    return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
inline double norm(const Vec3& a) { return std::sqrt(dot(a, a)); }

thread_local std::string g_last_error;

// Runs f(begin, end, thread_index) over [0, n) in contiguous chunks.
template <class F>
void parallel_for(int64_t n, int nt, F f) {
    if (nt <= 1 || n < 1024) {
        f(int64_t(0), n, 0);
        return;
    }
    std::vector<std::thread> pool;
    int64_t chunk = (n + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
        int64_t b = t * chunk, e = std::min(n, b + chunk);
        if (b >= e) break;
        pool.emplace_back([=, &f] { f(b, e, t); });
    }
    for (auto& th : pool) th.join();
}
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

int cell_nfaces(int type) {
    switch (type) {
        case UCNS_TET: return 4;
        case UCNS_PYR: return 5;
        case UCNS_PRISM: return 5;
        case UCNS_HEX: return 6;
        default: return -1;
    }
}

const int* face_verts(int type, int lf, int* nv) {
    const int* row = type == UCNS_TET ? kTetFaces[lf]
                     : type == UCNS_PYR ? kPyrFaces[lf]
                     : type == UCNS_PRISM ? kPrismFaces[lf]
                                          : kHexFaces[lf];
    *nv = row[3] < 0 ? 3 : 4;
    return row;
}

namespace {

// ---------------------------------------------------------------- geometry

int cell_coords(const Mesh& m, int64_t c, Vec3* X) {
    int64_t p0 = m.cptr[c];
    int nv = int(m.cptr[c + 1] - p0);
    const double* x0 = &m.xyz[3 * m.cvtx[p0]];
    for (int k = 0; k < nv; ++k) {
        const double* x = &m.xyz[3 * m.cvtx[p0 + k]];
        for (int a = 0; a < 3; ++a) {
            double L = m.period[a];
            X[k][a] = L > 0 ? x[a] - L * std::nearbyint((x[a] - x0[a]) / L) : x[a];
        }
    }
    return nv;
}

void wrap(const Mesh& m, Vec3& d) {
    for (int a = 0; a < 3; ++a)
        if (m.period[a] > 0) d[a] -= m.period[a] * std::nearbyint(d[a] / m.period[a]);
}

// Sub-tetrahedra of the cell's geometric definition: apex at the vertex
// average, base triangles on the faces (quadrilaterals fanned about their
// vertex average).
int subtets(const Mesh& m, int64_t c, std::array<Vec3, 4>* T) {
    Vec3 X[8];
    int nv = cell_coords(m, c, X), type = m.type[c];
    Vec3 apex{0, 0, 0};
    for (int k = 0; k < nv; ++k) apex = apex + (1.0 / nv) * X[k];
    int nt = 0;
    for (int lf = 0; lf < cell_nfaces(type); ++lf) {
        int fnv;
        const int* fv = face_verts(type, lf, &fnv);
        if (fnv == 3) {
            T[nt++] = {apex, X[fv[0]], X[fv[1]], X[fv[2]]};
        } else {
            Vec3 fc = 0.25 * (X[fv[0]] + X[fv[1]] + X[fv[2]] + X[fv[3]]);
            for (int j = 0; j < 4; ++j) T[nt++] = {apex, X[fv[j]], X[fv[(j + 1) & 3]], fc};
        }
    }
    return nt;
}

// Grundmann-Moeller rule of degree 2s+1 on the reference tetrahedron
// (barycentric points, weights summing to 1): A. Grundmann, H. M. Moeller,
// SIAM J. Numer. Anal. 15 (1978).
struct SimplexRule {
    std::vector<std::array<double, 4>> bary;
    std::vector<double> w;
};

SimplexRule grundmann_moeller(int s) {
    SimplexRule r;
    const int n = 3, d = 2 * s + 1;
    double wsum = 0;
    for (int i = 0; i <= s; ++i) {
        double fact_i = std::tgamma(i + 1.0), fact = std::tgamma(double(d + n - i) + 1.0);
        double w = ((i & 1) ? -1.0 : 1.0) * std::ldexp(1.0, -2 * s) * std::pow(double(d + n - 2 * i), d) /
                   (fact_i * fact);
        int tot = s - i;
        double den = d + n - 2 * i;
        for (int b0 = 0; b0 <= tot; ++b0)
            for (int b1 = 0; b1 <= tot - b0; ++b1)
                for (int b2 = 0; b2 <= tot - b0 - b1; ++b2) {
                    int b3 = tot - b0 - b1 - b2;
                    r.bary.push_back({(2 * b0 + 1) / den, (2 * b1 + 1) / den, (2 * b2 + 1) / den, (2 * b3 + 1) / den});
                    r.w.push_back(w * 6.0);  // reference tet volume 1/6
                    wsum += w * 6.0;
                }
    }
    (void)wsum;
    return r;
}

// Gauss-Legendre nodes/weights on [0,1] (closed forms, ascending nodes).
void gauss01(int n, double* x, double* w) {
    if (n == 1) {
        x[0] = 0.5;
        w[0] = 1.0;
    } else if (n == 2) {
        double t = 0.5 / std::sqrt(3.0);
        x[0] = 0.5 - t, x[1] = 0.5 + t;
        w[0] = w[1] = 0.5;
    } else if (n == 3) {
        double t = 0.5 * std::sqrt(0.6);
        x[0] = 0.5 - t, x[1] = 0.5, x[2] = 0.5 + t;
        w[0] = w[2] = 5.0 / 18.0, w[1] = 8.0 / 18.0;
    } else {  // n == 4
        double a = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(1.2)), b = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(1.2));
        double wa = (18.0 + std::sqrt(30.0)) / 72.0, wb = (18.0 - std::sqrt(30.0)) / 72.0;
        x[0] = 0.5 - 0.5 * b, x[1] = 0.5 - 0.5 * a, x[2] = 0.5 + 0.5 * a, x[3] = 0.5 + 0.5 * b;
        w[0] = wb, w[1] = wa, w[2] = wa, w[3] = wb;
    }
}

// ------------------------------------------------------------------- faces

struct FaceKey {
    int64_t v[4];
    bool operator==(const FaceKey& o) const { return std::memcmp(v, o.v, sizeof v) == 0; }
};
struct FaceKeyHash {
    size_t operator()(const FaceKey& k) const {
        uint64_t h = 1469598103934665603ull;
        for (int i = 0; i < 4; ++i) {
            h ^= uint64_t(k.v[i]) + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
        }
        return size_t(h);
    }
};

FaceKey make_key(const int64_t* ids, int n) {
    FaceKey k;
    for (int i = 0; i < 4; ++i) k.v[i] = i < n ? ids[i] : -1;
    std::sort(k.v, k.v + n);
    return k;
}

int build_faces(Mesh& m) {
    std::unordered_map<FaceKey, int64_t, FaceKeyHash> seen;
    seen.reserve(size_t(m.nc) * 4);
    m.c2f.assign(size_t(m.nc) * kMaxFaces, -1);
    std::vector<int64_t> fc;
    std::vector<int> lf2;
    for (int64_t c = 0; c < m.nc; ++c) {
        int type = m.type[c];
        for (int lf = 0; lf < cell_nfaces(type); ++lf) {
            int fnv;
            const int* fv = face_verts(type, lf, &fnv);
            int64_t ids[4];
            for (int j = 0; j < fnv; ++j) ids[j] = m.cvtx[m.cptr[c] + fv[j]];
            FaceKey key = make_key(ids, fnv);
            auto it = seen.find(key);
            if (it == seen.end()) {
                int64_t f = int64_t(fc.size() / 2);
                seen.emplace(key, f);
                fc.push_back(c);
                fc.push_back(-1);
                lf2.push_back(lf);
                lf2.push_back(-1);
                m.c2f[c * kMaxFaces + lf] = int32_t(2 * f);
            } else {
                int64_t f = it->second;
                if (fc[2 * f + 1] != -1) {
                    set_error("non-manifold face (three cells) at cell " + std::to_string(c));
                    return UCNS_EMESH;
                }
                if (fc[2 * f] == c) {
                    set_error("cell " + std::to_string(c) + " meets itself through a face");
                    return UCNS_EMESH;
                }
                fc[2 * f + 1] = c;
                lf2[2 * f + 1] = lf;
                m.c2f[c * kMaxFaces + lf] = int32_t(2 * f + 1);
            }
        }
    }
    m.nf = int64_t(fc.size() / 2);
    if (m.nf * 2 >= (int64_t(1) << 31)) {
        set_error("too many faces for 32-bit face indices");
        return UCNS_EINVAL;
    }
    m.fcell = std::move(fc);
    m.flf = std::move(lf2);
    return UCNS_OK;
}

int match_boundaries(Mesh& m, const ucns_mesh_desc* d) {
    std::unordered_map<FaceKey, int, FaceKeyHash> tags;
    for (int64_t b = 0; b < d->n_bface; ++b) {
        int n = int(d->bface_ptr[b + 1] - d->bface_ptr[b]);
        if (n < 3 || n > 4) {
            set_error("boundary face with " + std::to_string(n) + " vertices");
            return UCNS_EINVAL;
        }
        tags[make_key(d->bface_vtx + d->bface_ptr[b], n)] = d->bface_tag[b];
    }
    m.nbnd = 0;
    for (int64_t f = 0; f < m.nf; ++f) {
        if (m.fcell[2 * f + 1] != -1) continue;
        int64_t c = m.fcell[2 * f];
        int fnv;
        const int* fv = face_verts(m.type[c], m.flf[2 * f], &fnv);
        int64_t ids[4];
        for (int j = 0; j < fnv; ++j) ids[j] = m.cvtx[m.cptr[c] + fv[j]];
        auto it = tags.find(make_key(ids, fnv));
        if (it == tags.end() || it->second < 1 || it->second > 7) {
            set_error("unmatched face of cell " + std::to_string(c) + " (no neighbour and no boundary tag)");
            return UCNS_EMESH;
        }
        m.fcell[2 * f + 1] = -1 - it->second;
        ++m.nbnd;
    }
    return UCNS_OK;
}

void face_geometry(Mesh& m) {
    const int Q = m.qmax;
    m.farea.assign(m.nf, 0);
    m.fnrm.assign(3 * m.nf, 0);
    m.fcen.assign(3 * m.nf, 0);
    m.fqp.assign(size_t(m.nf) * Q * 3, 0);
    m.fqw.assign(size_t(m.nf) * Q, 0);
    m.fshift.assign(3 * m.nf, 0);
    m.fnq.assign(m.nf, 0);
    double gx[4], gw[4];
    gauss01(m.order, gx, gw);
    for (int64_t f = 0; f < m.nf; ++f) {
        int64_t cL = m.fcell[2 * f];
        Vec3 X[8];
        cell_coords(m, cL, X);
        int fnv;
        const int* fv = face_verts(m.type[cL], m.flf[2 * f], &fnv);
        Vec3 V[4];
        for (int j = 0; j < fnv; ++j) V[j] = X[fv[j]];
        Vec3 S = fnv == 3 ? 0.5 * cross(V[1] - V[0], V[2] - V[0]) : 0.5 * cross(V[2] - V[0], V[3] - V[1]);
        double A = norm(S);
        m.farea[f] = A;
        Vec3 cen{0, 0, 0};
        for (int j = 0; j < fnv; ++j) cen = cen + (1.0 / fnv) * V[j];
        for (int a = 0; a < 3; ++a) {
            m.fnrm[3 * f + a] = S[a] / A;
            m.fcen[3 * f + a] = cen[a];
        }
        double* qp = &m.fqp[size_t(f) * Q * 3];
        double* qw = &m.fqw[size_t(f) * Q];
        if (fnv == 3) {
            // degree-2 rule: barycentric (2/3, 1/6, 1/6) and its rotations
            for (int q = 0; q < 3; ++q) {
                Vec3 p = (1.0 / 6.0) * (V[0] + V[1] + V[2]) + 0.5 * V[q];
                for (int a = 0; a < 3; ++a) qp[3 * q + a] = p[a];
                qw[q] = 1.0 / 3.0;
            }
            m.fnq[f] = 3;
        } else {
            int n = m.order;
            double tot = 0;
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    double s = gx[i], t = gx[j];
                    Vec3 p = ((1 - s) * (1 - t)) * V[0] + (s * (1 - t)) * V[1] + (s * t) * V[2] + ((1 - s) * t) * V[3];
                    Vec3 xs = (1 - t) * (V[1] - V[0]) + t * (V[2] - V[3]);
                    Vec3 xt = (1 - s) * (V[3] - V[0]) + s * (V[2] - V[1]);
                    int q = i + n * j;
                    for (int a = 0; a < 3; ++a) qp[3 * q + a] = p[a];
                    qw[q] = gw[i] * gw[j] * norm(cross(xs, xt));
                    tot += qw[q];
                }
            for (int q = 0; q < n * n; ++q) qw[q] /= tot;
            m.fnq[f] = n * n;
        }
        int64_t cR = m.fcell[2 * f + 1];
        if (cR >= 0) {
            Vec3 XR[8];
            int nvR = cell_coords(m, cR, XR);
            int64_t g = m.cvtx[m.cptr[cL] + fv[0]];
            for (int k = 0; k < nvR; ++k)
                if (m.cvtx[m.cptr[cR] + k] == g) {
                    for (int a = 0; a < 3; ++a) {
                        double L = m.period[a], dd = V[0][a] - XR[k][a];
                        m.fshift[3 * f + a] = L > 0 ? L * std::nearbyint(dd / L) : 0.0;
                    }
                    break;
                }
        }
    }
}

// ----------------------------------------------------------- cell geometry

inline int mom_index(int D, int a, int b, int c) { return (a * (D + 1) + b) * (D + 1) + c; }

void cell_geometry(Mesh& m, int nt) {
    m.vol.assign(m.nc, 0);
    m.cen.assign(3 * m.nc, 0);
    m.hb.assign(m.nc, 0);
    m.hdt.assign(m.nc, 0);
    const int D = m.mom_deg;
    m.nmom = (D + 1) * (D + 1) * (D + 1);
    m.moments.assign(size_t(m.nc) * m.nmom, 0);
    SimplexRule gm = grundmann_moeller((D + 1) / 2);  // degree 2s+1 >= D
    parallel_for(m.nc, nt, [&](int64_t b, int64_t e, int) {
        std::array<Vec3, 4> T[24];
        std::vector<double> pw(D + 1);
        for (int64_t c = b; c < e; ++c) {
            int n = subtets(m, c, T);
            double V = 0;
            Vec3 C{0, 0, 0};
            double vt[24];
            for (int t = 0; t < n; ++t) {
                vt[t] = dot(T[t][1] - T[t][0], cross(T[t][2] - T[t][0], T[t][3] - T[t][0])) / 6.0;
                V += vt[t];
                C = C + (vt[t] * 0.25) * (T[t][0] + T[t][1] + T[t][2] + T[t][3]);
            }
            C = (1.0 / V) * C;
            m.vol[c] = V;
            for (int a = 0; a < 3; ++a) m.cen[3 * c + a] = C[a];
            double* M = &m.moments[size_t(c) * m.nmom];
            for (int t = 0; t < n; ++t)
                for (size_t q = 0; q < gm.w.size(); ++q) {
                    const auto& l = gm.bary[q];
                    Vec3 y = (l[0] * T[t][0] + l[1] * T[t][1] + l[2] * T[t][2] + l[3] * T[t][3]) - C;
                    double w = gm.w[q] * vt[t];
                    double px[8], py[8], pz[8];
                    px[0] = py[0] = pz[0] = 1.0;
                    for (int k = 1; k <= D; ++k) {
                        px[k] = px[k - 1] * y[0];
                        py[k] = py[k - 1] * y[1];
                        pz[k] = pz[k - 1] * y[2];
                    }
                    for (int a = 0; a <= D; ++a)
                        for (int bb = 0; bb <= D - a; ++bb)
                            for (int cc = 0; cc <= D - a - bb; ++cc) M[mom_index(D, a, bb, cc)] += w * px[a] * py[bb] * pz[cc];
                }
            Vec3 X[8];
            int nv = cell_coords(m, c, X);
            double h = 0, S = 0;
            for (int k = 0; k < nv; ++k) h = std::max(h, norm(X[k] - C));
            m.hb[c] = h;
            for (int lf = 0; lf < cell_nfaces(m.type[c]); ++lf) S += m.farea[m.c2f[c * kMaxFaces + lf] >> 1];
            m.hdt[c] = 6.0 * V / S;
        }
    });
    m.total_vol = 0;
    for (int64_t c = 0; c < m.nc; ++c) m.total_vol += m.vol[c];
}

// ----------------------------------------------------------------- stencils

struct Cand {
    double dist;
    int64_t id;
};

// Stencil rule (the paper cites the selection algorithm without giving it):
// vertex-neighbour layers until >= 2 Mc candidates (at least 2, at most
// max_layers layers); central = Mc = round(stencil_factor K(r,3)) nearest
// centroids (periodic minimum image)
// closed over distance ties within 1e-9; directional = up to 8 nearest
// candidates inside the closed cone from the centroid through each face,
// closed over ties, dropped below 4.
int build_stencils(Mesh& m, int nt) {
    const int Mc = int(std::lround(m.stencil_factor * (m.K + 1)));
    std::vector<int64_t> v2c_ptr(m.nv + 1, 0), v2c(m.cptr[m.nc]);
    for (int64_t p = 0; p < m.cptr[m.nc]; ++p) v2c_ptr[m.cvtx[p] + 1]++;
    for (int64_t v = 0; v < m.nv; ++v) v2c_ptr[v + 1] += v2c_ptr[v];
    {
        std::vector<int64_t> fill(v2c_ptr.begin(), v2c_ptr.end() - 1);
        for (int64_t c = 0; c < m.nc; ++c)
            for (int64_t p = m.cptr[c]; p < m.cptr[c + 1]; ++p) v2c[fill[m.cvtx[p]]++] = c;
    }
    m.ncen.assign(m.nc, 0);
    m.navail.assign(m.nc, 0);
    m.cand.assign(size_t(m.nc) * kMaxCentral, -1);
    m.cdist.assign(size_t(m.nc) * kMaxCentral, 0);
    m.ndir.assign(m.nc, 0);
    m.ndropped.assign(m.nc, 0);
    m.nds.assign(size_t(m.nc) * kMaxFaces, 0);
    m.dface.assign(size_t(m.nc) * kMaxFaces, -1);
    m.dir.assign(size_t(m.nc) * kMaxFaces * kMaxDir, -1);
    std::atomic<int> err{UCNS_OK};
    std::mutex emu;
    std::string emsg;
    parallel_for(m.nc, nt, [&](int64_t b, int64_t e, int) {
        std::vector<int64_t> stamp(m.nc, -1), list;
        std::vector<Cand> pool;
        for (int64_t c = b; c < e && err.load() == UCNS_OK; ++c) {
            list.clear();
            list.push_back(c);
            stamp[c] = c;
            size_t head = 0;
            for (int L = 1;; ++L) {
                size_t stop = list.size();
                for (; head < stop; ++head) {
                    int64_t cc = list[head];
                    for (int64_t p = m.cptr[cc]; p < m.cptr[cc + 1]; ++p) {
                        int64_t v = m.cvtx[p];
                        for (int64_t q = v2c_ptr[v]; q < v2c_ptr[v + 1]; ++q) {
                            int64_t nb = v2c[q];
                            if (stamp[nb] != c) {
                                stamp[nb] = c;
                                list.push_back(nb);
                            }
                        }
                    }
                }
                bool grew = list.size() > stop;
                if ((L >= 2 && int64_t(list.size()) - 1 >= 2 * Mc) || L >= m.max_layers || !grew) break;
            }
            pool.clear();
            Vec3 ci{m.cen[3 * c], m.cen[3 * c + 1], m.cen[3 * c + 2]};
            for (size_t k = 1; k < list.size(); ++k) {
                int64_t id = list[k];
                Vec3 d = Vec3{m.cen[3 * id], m.cen[3 * id + 1], m.cen[3 * id + 2]} - ci;
                wrap(m, d);
                pool.push_back({norm(d), id});
            }
            std::sort(pool.begin(), pool.end(), [](const Cand& x, const Cand& y) {
                return x.dist < y.dist || (x.dist == y.dist && x.id < y.id);
            });
            int n = std::min<int>(Mc, int(pool.size()));
            if (n < m.K) {
                std::lock_guard<std::mutex> g(emu);
                emsg = "cell " + std::to_string(c) + ": too few stencil candidates";
                err = UCNS_ERANK;
                break;
            }
            double lim = pool[n - 1].dist * (1.0 + 1e-9);
            while (n < int(pool.size()) && pool[n].dist <= lim) ++n;
            if (n > kMaxCentral) {
                std::lock_guard<std::mutex> g(emu);
                emsg = "cell " + std::to_string(c) + ": central stencil exceeds the cap";
                err = UCNS_EMESH;
                break;
            }
            m.ncen[c] = n;
            int na = std::min<int>(kMaxCentral, int(pool.size()));
            m.navail[c] = na;
            for (int k = 0; k < na; ++k) {
                m.cand[size_t(c) * kMaxCentral + k] = pool[k].id;
                m.cdist[size_t(c) * kMaxCentral + k] = pool[k].dist;
            }
            // directional sectors
            Vec3 X[8];
            cell_coords(m, c, X);
            int type = m.type[c], s = 0;
            for (int lf = 0; lf < cell_nfaces(type); ++lf) {
                int fnv;
                const int* fv = face_verts(type, lf, &fnv);
                Vec3 rel[4], fc{0, 0, 0}, pn[4];
                for (int j = 0; j < fnv; ++j) {
                    rel[j] = X[fv[j]] - ci;
                    fc = fc + (1.0 / fnv) * rel[j];
                }
                for (int j = 0; j < fnv; ++j) {
                    pn[j] = cross(rel[j], rel[(j + 1) % fnv]);
                    if (dot(pn[j], fc) < 0) pn[j] = -1.0 * pn[j];
                }
                int cnt = 0;
                double cut = -1;
                int64_t* out = &m.dir[(size_t(c) * kMaxFaces + s) * kMaxDir];
                for (const Cand& p : pool) {
                    Vec3 d = Vec3{m.cen[3 * p.id], m.cen[3 * p.id + 1], m.cen[3 * p.id + 2]} - ci;
                    wrap(m, d);
                    bool in = true;
                    for (int j = 0; j < fnv && in; ++j) in = dot(d, pn[j]) >= -1e-9 * p.dist * norm(pn[j]);
                    if (!in) continue;
                    if (cnt >= dir_target(m.kd) && p.dist > cut) break;
                    if (cnt >= kMaxDir) {
                        std::lock_guard<std::mutex> g(emu);
                        emsg = "cell " + std::to_string(c) + ": directional stencil overflow";
                        err = UCNS_EMESH;
                        break;
                    }
                    out[cnt++] = p.id;
                    if (cnt == dir_target(m.kd)) cut = p.dist * (1.0 + 1e-9);
                }
                if (cnt < dir_min(m.kd)) {
                    for (int k = 0; k < kMaxDir; ++k) out[k] = -1;
                    m.ndropped[c]++;
                    continue;
                }
                m.nds[c * kMaxFaces + s] = cnt;
                m.dface[c * kMaxFaces + s] = lf;
                ++s;
            }
            m.ndir[c] = s;
        }
    });
    if (err != UCNS_OK) {
        set_error(emsg);
        return err;
    }
    return UCNS_OK;
}

// ----------------------------------------------------------- least squares

// B = A^+ diag(w) for the (n x k) matrix A (row-major), via modified
// Gram-Schmidt with one re-orthogonalisation pass on the column-equilibrated
// matrix.  rcond = min |R_jj| / |R_11| of the equilibrated factor.  B is
// (k x n) row-major.  Returns false when a column is exactly dependent.
bool lsq_pinv(int n, int k, const double* A, const double* w, double* B, double* rcond) {
    double Q[kMaxCentral * kMaxK], R[kMaxK * kMaxK], sc[kMaxK];
    for (int j = 0; j < k; ++j) {
        double s = 0;
        for (int i = 0; i < n; ++i) s += A[i * k + j] * A[i * k + j];
        sc[j] = s > 0 ? 1.0 / std::sqrt(s) : 1.0;
        for (int i = 0; i < n; ++i) Q[i * k + j] = A[i * k + j] * sc[j];
    }
    std::fill(R, R + k * k, 0.0);
    for (int j = 0; j < k; ++j) {
        for (int pass = 0; pass < 2; ++pass)
            for (int l = 0; l < j; ++l) {
                double r = 0;
                for (int i = 0; i < n; ++i) r += Q[i * k + l] * Q[i * k + j];
                for (int i = 0; i < n; ++i) Q[i * k + j] -= r * Q[i * k + l];
                R[l * k + j] += r;
            }
        double nn = 0;
        for (int i = 0; i < n; ++i) nn += Q[i * k + j] * Q[i * k + j];
        nn = std::sqrt(nn);
        R[j * k + j] = nn;
        if (nn == 0) {
            *rcond = 0;
            return false;
        }
        for (int i = 0; i < n; ++i) Q[i * k + j] /= nn;
    }
    double r11 = std::fabs(R[0]), rmin = r11;
    for (int j = 1; j < k; ++j) rmin = std::min(rmin, std::fabs(R[j * k + j]));
    *rcond = rmin / r11;
    // B = D R^{-1} Q^T diag(w): back-substitute each column of Q^T.
    for (int i = 0; i < n; ++i) {
        double y[kMaxK];
        for (int j = k - 1; j >= 0; --j) {
            double s = Q[i * k + j];
            for (int l = j + 1; l < k; ++l) s -= R[j * k + l] * y[l];
            y[j] = s / R[j * k + j];
        }
        for (int j = 0; j < k; ++j) B[j * n + i] = sc[j] * y[j] * w[i];
    }
    return true;
}

// ---------------------------------------------------------------- operators

struct Monomials {
    int K;
    int e[kMaxK][3];
};

Monomials make_monomials(int r) {
    Monomials mo;
    int k = 0;
    for (int d = 1; d <= r; ++d)
        for (int a = d; a >= 0; --a)
            for (int b = d - a; b >= 0; --b) {
                mo.e[k][0] = a, mo.e[k][1] = b, mo.e[k][2] = d - a - b;
                ++k;
            }
    mo.K = k;
    return mo;
}

inline double binom(int n, int k) {
    static const double t[8][8] = {{1}, {1, 1}, {1, 2, 1}, {1, 3, 3, 1}, {1, 4, 6, 4, 1}, {1, 5, 10, 10, 5, 1},
                                   {1, 6, 15, 20, 15, 6, 1}, {1, 7, 21, 35, 35, 21, 7, 1}};
    return t[n][k];
}

// integral over cell m (translated so that its centroid sits at c_i + d) of
// the monomial ((x - c_i)/h)^e, from m's central moments.
double shifted_monomial_integral(const Mesh& m, int64_t cell, const int* e, const Vec3& d, double h) {
    const double* M = &m.moments[size_t(cell) * m.nmom];
    const int D = m.mom_deg;
    double s = 0;
    for (int a = 0; a <= e[0]; ++a)
        for (int b = 0; b <= e[1]; ++b)
            for (int c = 0; c <= e[2]; ++c)
                s += binom(e[0], a) * binom(e[1], b) * binom(e[2], c) * std::pow(d[0], e[0] - a) *
                     std::pow(d[1], e[1] - b) * std::pow(d[2], e[2] - c) * M[mom_index(D, a, b, c)];
    return s / std::pow(h, e[0] + e[1] + e[2]);
}

int build_operators(Mesh& m, int nt) {
    const int K = m.K, Q = m.qmax, NF = m.nfmax;
    Monomials mo = make_monomials(m.order);
    // operator padding: central by the max stencil size after rank extension
    m.mean.assign(size_t(m.nc) * K, 0);
    m.O.assign(size_t(m.nc) * K * K, 0);
    m.Phi.assign(size_t(m.nc) * NF * Q * K, 0);
    m.xi.assign(size_t(m.nc) * NF * Q * 3, 0);
    // central operators: stride = largest stencil before rank extension;
    // the rare extended cells go to an overflow map
    int stride0 = 0;
    for (int64_t c = 0; c < m.nc; ++c) stride0 = std::max(stride0, m.ncen[c]);
    std::vector<double> Bc_main(size_t(m.nc) * K * stride0, 0);
    std::unordered_map<int64_t, std::vector<double>> Bc_over;
    std::mutex over_mu;
    m.nd_max = 0;
    m.md_pad = 0;
    for (int64_t c = 0; c < m.nc; ++c) {
        m.nd_max = std::max(m.nd_max, m.ndir[c]);
        for (int s = 0; s < m.ndir[c]; ++s) m.md_pad = std::max(m.md_pad, m.nds[c * kMaxFaces + s]);
    }
    const int kd = m.kd;
    m.Bd.assign(size_t(m.nc) * std::max(1, m.nd_max) * kd * std::max(1, m.md_pad), 0);
    std::atomic<int> err{UCNS_OK};
    std::mutex emu;
    std::string emsg;
    parallel_for(m.nc, nt, [&](int64_t b, int64_t e, int) {
        double A[kMaxCentral * kMaxK], w[kMaxCentral], B[kMaxK * kMaxCentral];
        for (int64_t c = b; c < e && err.load() == UCNS_OK; ++c) {
            const double V = m.vol[c], h = m.hb[c];
            const double* M = &m.moments[size_t(c) * m.nmom];
            const int D = m.mom_deg;
            Vec3 ci{m.cen[3 * c], m.cen[3 * c + 1], m.cen[3 * c + 2]};
            double* mean = &m.mean[size_t(c) * K];
            for (int k = 0; k < K; ++k) {
                const int* ek = mo.e[k];
                mean[k] = M[mom_index(D, ek[0], ek[1], ek[2])] / (V * std::pow(h, ek[0] + ek[1] + ek[2]));
            }
            auto row = [&](int64_t id, int kk, double* out) {
                Vec3 d = Vec3{m.cen[3 * id], m.cen[3 * id + 1], m.cen[3 * id + 2]} - ci;
                wrap(m, d);
                for (int k = 0; k < kk; ++k)
                    out[k] = shifted_monomial_integral(m, id, mo.e[k], d, h) - mean[k] * m.vol[id];
            };
            // central stencil, extended shell by shell while rank deficient
            int n = m.ncen[c];
            const int64_t* cand = &m.cand[size_t(c) * kMaxCentral];
            const double* cd = &m.cdist[size_t(c) * kMaxCentral];
            int built = 0;
            while (true) {
                for (; built < n; ++built) {
                    row(cand[built], K, A + built * K);
                    w[built] = m.vol[cand[built]];
                }
                double rc;
                bool ok = lsq_pinv(n, K, A, w, B, &rc);
                // extended until well conditioned (|R_jj| / |R_11| >= 1e-6):
                // thin boundary-layer prism stencils otherwise reach
                // condition numbers near 1e7
                if (ok && rc >= 1e-6) break;
                if (n >= m.navail[c]) {
                    std::lock_guard<std::mutex> g(emu);
                    emsg = "cell " + std::to_string(c) + ": central stencil rank deficient";
                    err = UCNS_ERANK;
                    break;
                }
                double lim = cd[n] * (1.0 + 1e-9);
                while (n < m.navail[c] && cd[n] <= lim) ++n;
            }
            if (err.load() != UCNS_OK) break;
            m.ncen[c] = n;
            if (n <= stride0) {
                for (int k = 0; k < K; ++k)
                    for (int j = 0; j < n; ++j) Bc_main[(size_t(c) * K + k) * stride0 + j] = B[k * n + j];
            } else {
                std::lock_guard<std::mutex> g(over_mu);
                Bc_over[c].assign(B, B + size_t(K) * n);
            }
            // directional stencils (the first kd basis functions: linear at
            // P2/P3, quadratic at P4); one whose members cannot fix a
            // linear polynomial (all in one plane through the centroid,
            // as on thin boundary-layer cells: a column of A vanishes up to
            // rounding, which the solve's unit-norm column scaling would
            // hide) is dropped like a sector with too few candidates, the
            // later ones moving down a slot
            for (int s = 0; s < m.ndir[c];) {
                int nd = m.nds[c * kMaxFaces + s];
                int64_t* ids = &m.dir[(size_t(c) * kMaxFaces + s) * kMaxDir];
                for (int j = 0; j < nd; ++j) {
                    row(ids[j], kd, A + j * kd);
                    w[j] = m.vol[ids[j]];
                }
                double cmin = INFINITY, cmax = 0;
                for (int k = 0; k < 3; ++k) {
                    double cn = 0;
                    for (int j = 0; j < nd; ++j) cn += A[j * kd + k] * A[j * kd + k];
                    cmin = std::min(cmin, std::sqrt(cn));
                    cmax = std::max(cmax, std::sqrt(cn));
                }
                double rc;
                if (!lsq_pinv(nd, kd, A, w, B, &rc) || rc < 1e-9 || cmin < 1e-8 * cmax) {
                    for (int t = s; t + 1 < m.ndir[c]; ++t) {
                        m.nds[c * kMaxFaces + t] = m.nds[c * kMaxFaces + t + 1];
                        m.dface[c * kMaxFaces + t] = m.dface[c * kMaxFaces + t + 1];
                        std::copy_n(&m.dir[(size_t(c) * kMaxFaces + t + 1) * kMaxDir], kMaxDir,
                                    &m.dir[(size_t(c) * kMaxFaces + t) * kMaxDir]);
                    }
                    m.ndir[c]--;
                    m.ndropped[c]++;
                    continue;
                }
                for (int k = 0; k < kd; ++k)
                    for (int j = 0; j < nd; ++j)
                        m.Bd[((size_t(c) * m.nd_max + s) * kd + k) * m.md_pad + j] = B[k * nd + j];
                ++s;
            }
            // smoothness-indicator matrix:
            // O_kl = sum_{1<=|b|<=r} V^{2|b|/3-1} int D^b phi_k D^b phi_l dV
            double* O = &m.O[size_t(c) * K * K];
            for (int bi = 0; bi < K; ++bi) {
                const int* be = mo.e[bi];
                int ob = be[0] + be[1] + be[2];
                double scale = std::pow(V, 2.0 * ob / 3.0 - 1.0) / std::pow(h, 2 * ob);
                for (int k = 0; k < K; ++k) {
                    const int* ek = mo.e[k];
                    if (ek[0] < be[0] || ek[1] < be[1] || ek[2] < be[2]) continue;
                    double ck = 1;
                    for (int a = 0; a < 3; ++a)
                        for (int t = 0; t < be[a]; ++t) ck *= double(ek[a] - t);
                    for (int l = 0; l < K; ++l) {
                        const int* el = mo.e[l];
                        if (el[0] < be[0] || el[1] < be[1] || el[2] < be[2]) continue;
                        double cl = 1;
                        for (int a = 0; a < 3; ++a)
                            for (int t = 0; t < be[a]; ++t) cl *= double(el[a] - t);
                        int g0 = ek[0] + el[0] - 2 * be[0], g1 = ek[1] + el[1] - 2 * be[1], g2 = ek[2] + el[2] - 2 * be[2];
                        double integ = M[mom_index(D, g0, g1, g2)] / std::pow(h, g0 + g1 + g2);
                        O[k * K + l] += scale * ck * cl * integ;
                    }
                }
            }
            // basis at the cell's own face points (neighbour side: owner's
            // points moved into this cell's frame)
            for (int lf = 0; lf < cell_nfaces(m.type[c]); ++lf) {
                int32_t fs = m.c2f[c * kMaxFaces + lf];
                int64_t f = fs >> 1;
                int side = fs & 1;
                for (int q = 0; q < m.fnq[f]; ++q) {
                    Vec3 x;
                    for (int a = 0; a < 3; ++a)
                        x[a] = m.fqp[(size_t(f) * Q + q) * 3 + a] - (side ? m.fshift[3 * f + a] : 0.0);
                    Vec3 xi = (1.0 / h) * (x - ci);
                    for (int a = 0; a < 3; ++a) m.xi[((size_t(c) * NF + lf) * Q + q) * 3 + a] = xi[a];
                    double* phi = &m.Phi[((size_t(c) * NF + lf) * Q + q) * K];
                    for (int k = 0; k < K; ++k) {
                        const int* ek = mo.e[k];
                        phi[k] = std::pow(xi[0], ek[0]) * std::pow(xi[1], ek[1]) * std::pow(xi[2], ek[2]) - mean[k];
                    }
                }
            }
        }
    });
    if (err != UCNS_OK) {
        set_error(emsg);
        return err;
    }
    m.mc_pad = 0;
    m.mc_min = kMaxCentral;
    for (int64_t c = 0; c < m.nc; ++c) {
        m.mc_pad = std::max(m.mc_pad, m.ncen[c]);
        m.mc_min = std::min(m.mc_min, m.ncen[c]);
    }
    if (m.mc_pad == stride0) {
        m.Bc = std::move(Bc_main);
    } else {
        m.Bc.assign(size_t(m.nc) * K * m.mc_pad, 0);
        for (int64_t c = 0; c < m.nc; ++c)
            for (int k = 0; k < K; ++k)
                for (int j = 0; j < std::min(m.ncen[c], stride0); ++j)
                    m.Bc[(size_t(c) * K + k) * m.mc_pad + j] = Bc_main[(size_t(c) * K + k) * stride0 + j];
    }
    for (auto& kv : Bc_over) {
        int64_t c = kv.first;
        int n = m.ncen[c];
        for (int k = 0; k < K; ++k)
            for (int j = 0; j < n; ++j) m.Bc[(size_t(c) * K + k) * m.mc_pad + j] = kv.second[size_t(k) * n + j];
    }
    m.n_dropped_total = 0;
    for (int64_t c = 0; c < m.nc; ++c) m.n_dropped_total += m.ndropped[c];
    return UCNS_OK;
}

}  // namespace

// Least-squares gradient weights: grad W_i = sum_slots G_slot (W_slot - W_i),
// G = pinv(diag(s) D) diag(s) with rows d = the fdc offset seen from cell i
// (owner->neighbour, negated from the neighbour's side; boundary faces the
// mirrored centroid) and s = 1/|d|, i.e. weights 1/|d|^2.
static int build_gradient_weights(Mesh& m) {
    m.glsq.assign(size_t(m.nc) * kMaxFaces * 3, 0.0);
    for (int64_t c = 0; c < m.nc; ++c) {
        double D[kMaxFaces * 3], s[kMaxFaces], G[3 * kMaxFaces], rc = 0;
        int slot[kMaxFaces], n = 0;
        for (int lf = 0; lf < kMaxFaces; ++lf) {
            const int32_t fs = m.c2f[c * kMaxFaces + lf];
            if (fs < 0) continue;
            const int64_t f = fs >> 1;
            const double sg = (fs & 1) ? -1.0 : 1.0;
            double dd = 0;
            for (int a = 0; a < 3; ++a) {
                D[n * 3 + a] = sg * m.fdc[3 * f + a];
                dd += D[n * 3 + a] * D[n * 3 + a];
            }
            s[n] = 1.0 / std::sqrt(dd);
            for (int a = 0; a < 3; ++a) D[n * 3 + a] *= s[n];
            slot[n++] = lf;
        }
        if (n < 3 || !lsq_pinv(n, 3, D, s, G, &rc) || rc < 1e-10) {
            set_error("cell " + std::to_string(c) + ": least-squares gradient fit is singular");
            return UCNS_ERANK;
        }
        for (int j = 0; j < n; ++j)
            for (int a = 0; a < 3; ++a) m.glsq[(size_t(c) * kMaxFaces + slot[j]) * 3 + a] = G[a * n + j];
    }
    return UCNS_OK;
}

int build_mesh(const ucns_mesh_desc* d, const ucns_recon_opts* o, int n_threads, Mesh** out) {
    if (!d || !o || !out) {
        set_error("null argument");
        return UCNS_EINVAL;
    }
    if (o->order < 2 || o->order > 4) {
        set_error("order must be 2, 3 or 4");
        return UCNS_EINVAL;
    }
    if (d->n_cell <= 0 || d->n_vert <= 0 || !d->xyz || !d->type || !d->cell_ptr || !d->cell_vtx) {
        set_error("empty mesh description");
        return UCNS_EINVAL;
    }
    if (d->n_cell >= (int64_t(1) << 31)) {
        set_error("too many cells for 32-bit cell indices");
        return UCNS_EINVAL;
    }
    int nt = n_threads > 0 ? n_threads : int(std::max(1u, std::thread::hardware_concurrency()));
    auto* m = new Mesh();
    m->nv = d->n_vert;
    m->nc = d->n_cell;
    m->xyz.assign(d->xyz, d->xyz + 3 * d->n_vert);
    m->type.assign(d->type, d->type + d->n_cell);
    m->cptr.assign(d->cell_ptr, d->cell_ptr + d->n_cell + 1);
    m->cvtx.assign(d->cell_vtx, d->cell_vtx + m->cptr[m->nc]);
    for (int a = 0; a < 3; ++a) m->period[a] = d->period[a];
    m->order = o->order;
    m->K = (o->order + 1) * (o->order + 2) * (o->order + 3) / 6 - 1;
    // directional polynomials: linear for the third- and fourth-order
    // schemes, quadratic for the fifth (Sec. 2.2)
    m->kd = o->order >= 4 ? 9 : 3;
    m->lambda_c = o->lambda_c;
    m->eps = o->eps;
    m->max_layers = o->max_layers;
    m->stencil_factor = o->stencil_factor > 0 ? o->stencil_factor : 2.0;
    m->mom_deg = std::max(o->order, 2 * o->order - 2);
    bool has_quad = false, has_tri = false;
    m->nfmax = 0;
    for (int64_t c = 0; c < m->nc; ++c) {
        int t = m->type[c], nf = cell_nfaces(t);
        if (nf < 0 || m->cptr[c + 1] - m->cptr[c] != t) {
            set_error("cell " + std::to_string(c) + ": bad type or vertex count");
            delete m;
            return UCNS_EINVAL;
        }
        m->nfmax = std::max(m->nfmax, nf);
        for (int lf = 0; lf < nf; ++lf) {
            int fnv;
            face_verts(t, lf, &fnv);
            (fnv == 3 ? has_tri : has_quad) = true;
        }
    }
    if (o->order >= 4 && has_tri) {
        set_error("order 4 is built for meshes of quadrilateral faces only (the 3-point triangle rule is exact "
                  "to degree 2)");
        delete m;
        return UCNS_EINVAL;
    }
    m->qmax = std::max(has_quad ? o->order * o->order : 0, has_tri ? 3 : 0);
    for (int64_t c = 1; c < m->nc; ++c)
        if (m->type[c] != m->type[0]) m->uniform_type = false;
    int rc = build_faces(*m);
    if (rc == UCNS_OK) rc = match_boundaries(*m, d);
    if (rc != UCNS_OK) {
        delete m;
        return rc;
    }
    face_geometry(*m);
    cell_geometry(*m, nt);
    for (int64_t c = 0; c < m->nc; ++c)
        if (!(m->vol[c] > 0)) {
            set_error("cell " + std::to_string(c) + " has non-positive volume");
            delete m;
            return UCNS_EMESH;
        }
    // owner -> neighbour centroid offset (boundary: twice the normal distance)
    m->fdc.assign(3 * m->nf, 0);
    for (int64_t f = 0; f < m->nf; ++f) {
        int64_t cL = m->fcell[2 * f], cR = m->fcell[2 * f + 1];
        if (cR >= 0) {
            for (int a = 0; a < 3; ++a) m->fdc[3 * f + a] = m->cen[3 * cR + a] + m->fshift[3 * f + a] - m->cen[3 * cL + a];
        } else {
            double dn = 0;
            for (int a = 0; a < 3; ++a) dn += (m->fcen[3 * f + a] - m->cen[3 * cL + a]) * m->fnrm[3 * f + a];
            for (int a = 0; a < 3; ++a) m->fdc[3 * f + a] = 2.0 * dn * m->fnrm[3 * f + a];
        }
    }
    rc = build_gradient_weights(*m);
    if (rc == UCNS_OK) rc = build_stencils(*m, nt);
    if (rc == UCNS_OK) rc = build_operators(*m, nt);
    if (rc != UCNS_OK) {
        delete m;
        return rc;
    }
    *out = m;
    return UCNS_OK;
}

}  // namespace ucns

namespace ucns {

// ------------------------------------------------------------------ packing
// Device arena of one precision: every per-cell array is cell-fastest
// ([entry][n_cell]) so that one thread per cell reads coalesced; stencil
// members are listed in ascending cell id (operator columns permuted alike)
// so that neighbouring threads gather from nearby cells.
namespace {
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <class T>
void fill_arena(const Mesh& m, const Arena& a, unsigned char* base) {
    const int64_t nc = m.nc, nf = m.nf;
    const int K = m.K, Q = m.qmax, NF = m.nfmax, MC = m.mc_pad, ND = std::max(1, m.nd_max), MD = std::max(1, m.md_pad);
    const int KD = m.kd;
    auto* sten_c = reinterpret_cast<int32_t*>(base + a.sten_c);
    auto* Bc = reinterpret_cast<T*>(base + a.Bc);
    auto* ndir = reinterpret_cast<uint8_t*>(base + a.ndir);
    auto* sten_d = reinterpret_cast<int32_t*>(base + a.sten_d);
    auto* Bd = reinterpret_cast<T*>(base + a.Bd);
    auto* O = reinterpret_cast<T*>(base + a.O);
    auto* xi = reinterpret_cast<T*>(base + a.xi);
    auto* pmean = reinterpret_cast<T*>(base + a.pmean);
    auto* c2f = reinterpret_cast<int32_t*>(base + a.c2f);
    auto* cnq = reinterpret_cast<uint8_t*>(base + a.cnq);
    auto* vol = reinterpret_cast<double*>(base + a.vol);
    auto* hdt = reinterpret_cast<double*>(base + a.hdt);
    auto* fcell = reinterpret_cast<int32_t*>(base + a.fcell);
    auto* flf = reinterpret_cast<uint8_t*>(base + a.flf);
    auto* fnrm = reinterpret_cast<T*>(base + a.fnrm);
    auto* farea = reinterpret_cast<T*>(base + a.farea);
    auto* fw = reinterpret_cast<T*>(base + a.fw);
    auto* fdc = reinterpret_cast<T*>(base + a.fdc);
    auto* fnq = reinterpret_cast<uint8_t*>(base + a.fnq);
    auto* nbr = reinterpret_cast<int32_t*>(base + a.nbr);
    auto* ndc = reinterpret_cast<T*>(base + a.ndc);
    auto* hb = reinterpret_cast<T*>(base + a.hb);
    auto* ncen = reinterpret_cast<uint8_t*>(base + a.ncen);
    auto* glsq = reinterpret_cast<T*>(base + a.glsq);
    auto* ggw = reinterpret_cast<T*>(base + a.ggw);
    for (int64_t c = 0; c < nc; ++c) {
        hb[c] = T(m.hb[c]);
        for (int lf = 0; lf < NF; ++lf)
            for (int k = 0; k < 3; ++k) glsq[(size_t(lf) * 3 + k) * nc + c] = T(m.glsq[(size_t(c) * kMaxFaces + lf) * 3 + k]);
        ncen[c] = uint8_t(m.ncen[c]);
        for (int lf = 0; lf < NF; ++lf) {
            const int32_t fs = m.c2f[c * kMaxFaces + lf];
            int32_t j = -1;
            double d[3] = {0, 0, 0}, w[3] = {0, 0, 0};
            if (fs >= 0) {
                const int64_t f = fs >> 1, side = fs & 1;
                const int64_t other = m.fcell[2 * f + (1 - side)];
                j = int32_t(other);  // a boundary face keeps its negative tag
                if (other >= 0)
                    for (int k = 0; k < 3; ++k) d[k] = (side ? -1.0 : 1.0) * m.fdc[3 * f + k];
                const double s = (side ? -0.5 : 0.5) * m.farea[f] / m.vol[c];
                for (int k = 0; k < 3; ++k) w[k] = s * m.fnrm[3 * f + k];
            }
            nbr[size_t(lf) * nc + c] = j;
            for (int k = 0; k < 3; ++k) {
                ndc[(size_t(lf) * 3 + k) * nc + c] = T(d[k]);
                ggw[(size_t(lf) * 3 + k) * nc + c] = T(w[k]);
            }
        }
    }
    std::vector<int> perm(kMaxCentral);
    for (int64_t c = 0; c < nc; ++c) {
        const int64_t* ids = &m.cand[size_t(c) * kMaxCentral];
        int n = m.ncen[c];
        for (int j = 0; j < n; ++j) perm[j] = j;
        std::sort(perm.begin(), perm.begin() + n, [&](int x, int y) { return ids[x] < ids[y]; });
        for (int j = 0; j < MC; ++j) {
            sten_c[size_t(j) * nc + c] = j < n ? int32_t(ids[perm[j]]) : int32_t(c);
            for (int k = 0; k < K; ++k)  // member-major rows: (j, k) at (j K + k) nc
                Bc[(size_t(j) * K + k) * nc + c] = j < n ? T(m.Bc[(size_t(c) * K + k) * MC + perm[j]]) : T(0);
        }
        ndir[c] = uint8_t(m.ndir[c]);
        for (int s = 0; s < ND; ++s) {
            int nd = s < m.ndir[c] ? m.nds[c * kMaxFaces + s] : 0;
            const int64_t* dids = &m.dir[(size_t(c) * kMaxFaces + s) * kMaxDir];
            for (int j = 0; j < nd; ++j) perm[j] = j;
            std::sort(perm.begin(), perm.begin() + nd, [&](int x, int y) { return dids[x] < dids[y]; });
            for (int j = 0; j < MD; ++j) {
                sten_d[(size_t(s) * MD + j) * nc + c] = j < nd ? int32_t(dids[perm[j]]) : int32_t(c);
                for (int k = 0; k < KD; ++k)  // member-major rows: (s, j, k) at ((s MD + j) kd + k) nc
                    Bd[((size_t(s) * MD + j) * KD + k) * nc + c] =
                        j < nd ? T(m.Bd[((size_t(c) * m.nd_max + s) * KD + k) * m.md_pad + perm[j]]) : T(0);
            }
        }
        int t = 0;
        for (int k = 0; k < K; ++k)
            for (int l = k; l < K; ++l) O[size_t(t++) * nc + c] = T(m.O[(size_t(c) * K + k) * K + l]);
        for (int k = 0; k < K; ++k) pmean[size_t(k) * nc + c] = T(m.mean[size_t(c) * K + k]);
        for (int lf = 0; lf < NF; ++lf) {
            const int32_t fs = m.c2f[c * kMaxFaces + lf];
            c2f[size_t(lf) * nc + c] = fs;
            cnq[size_t(lf) * nc + c] = fs >= 0 ? uint8_t(m.fnq[fs >> 1]) : 0;
            for (int q = 0; q < Q; ++q)
                for (int d = 0; d < 3; ++d)
                    xi[((size_t(lf) * Q + q) * 3 + d) * nc + c] = T(m.xi[((size_t(c) * NF + lf) * Q + q) * 3 + d]);
        }
        vol[c] = m.vol[c];
        hdt[c] = m.hdt[c];
    }
    for (int64_t f = 0; f < nf; ++f) {
        fcell[2 * f] = int32_t(m.fcell[2 * f]);
        fcell[2 * f + 1] = int32_t(m.fcell[2 * f + 1]);
        for (int side = 0; side < 2; ++side) flf[2 * f + side] = m.flf[2 * f + side] >= 0 ? uint8_t(m.flf[2 * f + side]) : 0xff;
        for (int a = 0; a < 3; ++a) {
            fnrm[3 * f + a] = T(m.fnrm[3 * f + a]);
            fdc[3 * f + a] = T(m.fdc[3 * f + a]);
        }
        farea[f] = T(m.farea[f]);
        for (int q = 0; q < Q; ++q) fw[size_t(f) * Q + q] = T(m.fqw[size_t(f) * Q + q]);
        fnq[f] = uint8_t(m.fnq[f]);
    }
}
}  // namespace

int pack_arena(const Mesh& m, int precision, Arena& a, std::vector<unsigned char>* image) {
    const size_t ts = precision == UCNS_F32 ? 4 : 8;
    const size_t nc = size_t(m.nc), nf = size_t(m.nf);
    const size_t K = m.K, Q = m.qmax, NF = m.nfmax, MC = m.mc_pad, ND = std::max(1, m.nd_max),
                 MD = std::max(1, m.md_pad);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    a.sten_c = take(4 * MC * nc);
    a.Bc = take(ts * K * MC * nc);
    a.ndir = take(nc);
    a.sten_d = take(4 * ND * MD * nc);
    a.Bd = take(ts * ND * m.kd * MD * nc);
    a.O = take(ts * K * (K + 1) / 2 * nc);
    a.xi = take(ts * NF * Q * 3 * nc);
    a.pmean = take(ts * K * nc);
    a.c2f = take(4 * NF * nc);
    a.cnq = take(NF * nc);
    a.vol = take(8 * nc);
    a.hdt = take(8 * nc);
    a.fcell = take(8 * nf);
    a.flf = take(2 * nf);
    a.fnrm = take(ts * 3 * nf);
    a.farea = take(ts * nf);
    a.fw = take(ts * Q * nf);
    a.fdc = take(ts * 3 * nf);
    a.fnq = take(nf);
    a.nbr = take(4 * NF * nc);
    a.ndc = take(ts * NF * 3 * nc);
    a.hb = take(ts * nc);
    a.ncen = take(nc);
    a.glsq = take(ts * NF * 3 * nc);
    a.ggw = take(ts * NF * 3 * nc);
    a.ustage = take(m.order == 4 ? 64 * nc : 0);  // scratch, written per reconstruction call
    a.bytes = off;
    if (image) {
        image->assign(a.bytes, 0);
        if (precision == UCNS_F32)
            fill_arena<float>(m, a, image->data());
        else
            fill_arena<double>(m, a, image->data());
    }
    return UCNS_OK;
}

}  // namespace ucns
