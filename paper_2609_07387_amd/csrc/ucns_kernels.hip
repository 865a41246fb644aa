// libucns device path for gfx950 (CDNA4): reconstruction, gradients, face
// fluxes, residual gather, SSP-RK3 stage, time step and diagnostics, plus the
// C-ABI entry points (declared in include/ucns.h).
//
// Method: Sec. 2.2 of the UCNS3D v4 paper (eqs. lsq_system, cwenoz_poly,
// cwenoz_weights, viscous_gradient_penalty, fv_update) with the per-stage
// order of its time-step algorithm (Algorithm 1).
//
// Layout: per-cell operators and the point states each cell writes are
// cell-fastest ([entry][n_cell]) so that one thread per cell streams them
// coalesced; face geometry and face fluxes are face-major.  The
// residual is a per-cell gather of single-valued face fluxes (no atomics),
// and the two reductions (dt, kinetic energy) use a fixed block count and a
// fixed tree, so every result is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <type_traits>
#include <mutex>
#include <vector>

#include "ucns_internal.hpp"

namespace ucns {
const char* last_error_cstr();
}

using namespace ucns;

namespace {

constexpr int kBlock = 256;
constexpr int kRedBlocks = 1024;  // fixed grid of the deterministic reductions

// The dispatcher hands workgroups to the eight XCDs round robin (block b runs
// on XCD b mod 8).  Renumbered this way, each XCD takes one contiguous range
// of blocks, so a cell's stencil neighbours and the face slots that adjacent
// cells both write mostly live in the same L2.  A bijection on [0, gridDim).
__device__ __forceinline__ int64_t xcd_block() {
    const uint32_t b = blockIdx.x, nb = gridDim.x;
    const uint32_t x = b & 7u, i = b >> 3, q = nb >> 3, r = nb & 7u;
    return int64_t(x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

template <class T>
struct PhysT {
    T gamma, gm1, gM2, mu, kappa, pr;  // gM2 = gamma M^2
    int viscous, flux;
};

template <class T>
struct BcT {
    int kind[8];
    T state[8][5];
};

template <class T>
PhysT<T> make_phys(const ucns_phys* p) {
    PhysT<T> o;
    o.gamma = T(p->gamma);
    o.gm1 = T(p->gamma - 1.0);
    o.gM2 = T(p->gamma * p->mach * p->mach);
    double mu = p->reynolds > 0 ? 1.0 / p->reynolds : 0.0;
    o.mu = T(mu);
    o.kappa = T(p->viscous ? mu / ((p->gamma - 1.0) * p->mach * p->mach * p->prandtl) : 0.0);
    o.pr = T(p->prandtl);
    o.viscous = p->viscous;
    o.flux = p->flux;
    return o;
}

template <class T>
BcT<T> make_bc(const ucns_bc* b) {
    BcT<T> o;
    for (int t = 0; t < 8; ++t) {
        o.kind[t] = b ? b->kind[t] : UCNS_BC_TRANSMISSIVE;
        for (int v = 0; v < 5; ++v) o.state[t][v] = b ? T(b->state[t][v]) : T(0);
    }
    return o;
}

// ------------------------------------------------------------ reconstruction

template <class T>
struct ReconArgs {
    const double* U;
    int64_t nc;
    const int32_t* sten_c;
    const T* Bc;
    int MC;
    int MCmin;  // smallest central stencil (MC when all cells have MC members)
    const uint8_t* ndir;
    const int32_t* sten_d;
    const T* Bd;
    int ND;       // directional stencil slots per cell (cells with fewer pad with zero operators)
    int MD;       // padded directional stencil size
    const T* O;
    const T* xi;     // face points in each cell's scaled frame [lf][q][3][nc]
    const T* pmean;  // cell means of the scaled monomials [K][nc]
    const uint8_t* cnq;  // Gauss points of each face slot [lf][nc] (0: no face)
    int Q, NF;
    const uint8_t* gate;
    T* fs;
    uint8_t* flags;
    float* label;
    T lam_c, eps, gm1;
    // troubled-cell gate (network inside the kernel) and its features
    const unsigned char* mlp;  // packed network image (ucns_mlp_pack)
    uint8_t* mask_out;
    const int32_t* nbr;
    const T* ndc;
    const T* hb;
    const uint8_t* ncen;
    double* ustage;  // P4: the state staged [cell][8] (scratch in the arena)
    // Green-Gauss gradients of the same state in the same pass (null: none);
    // the boundary table in device memory (null: every boundary transmissive)
    T* gradW;
    const T* ggw;
    const T* glsq;
    const ucns_bc* bcd;
    T gM2;
};

template <class T, bool LSQ>
__device__ void cell_gradient(const ReconArgs<T>& A, int64_t c, const double* ui);

__device__ __forceinline__ int tri_index(int K, int k, int l) { return k * K - (k * (k - 1)) / 2 + (l - k); }

#include "mlp_kernels.hpp"
#include "recon_kernel.hpp"
#include "recon_p4.hpp"

// ------------------------------------------------------------------ physics

template <class T>
__device__ __forceinline__ T pressure(const PhysT<T>& P, const T* u) {
    return P.gm1 * (u[4] - T(0.5) * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0]);
}

// Primitive quantities of one point state, formed once per Gauss point and
// shared by the convective and viscous fluxes (one reciprocal of the density
// instead of a division in every formula).
// Reciprocal, quotient and square root of the flux kernels: FP32 takes the hardware
// instructions (about 1 ulp) in place of the correctly rounded sequences, a
// fraction of the variant's rounding budget; FP64 stays exact.
template <class T>
__device__ __forceinline__ T rcp(T x) {
    if constexpr (sizeof(T) == 4)
        return __builtin_amdgcn_rcpf(x);
    else
        return T(1) / x;
}
template <class T>
__device__ __forceinline__ T fdiv(T a, T b) {
    if constexpr (sizeof(T) == 4)
        return a * __builtin_amdgcn_rcpf(b);
    else
        return a / b;
}
template <class T>
__device__ __forceinline__ T fsqrt(T x) {
    if constexpr (sizeof(T) == 4)
        return __builtin_amdgcn_sqrtf(x);
    else
        return sqrt(x);
}

template <class T>
struct Prim {
    T r, ir, u[3], un, p, c, E;
};

template <class T>
__device__ __forceinline__ Prim<T> prim(const PhysT<T>& P, const T* U, const T* n) {
    Prim<T> q;
    q.r = U[0];
    q.ir = rcp(U[0]);
#pragma unroll
    for (int a = 0; a < 3; ++a) q.u[a] = U[1 + a] * q.ir;
    q.un = q.u[0] * n[0] + q.u[1] * n[1] + q.u[2] * n[2];
    q.E = U[4];
    q.p = P.gm1 * (U[4] - T(0.5) * q.r * (q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2]));
    q.c = fsqrt(P.gamma * q.p * q.ir);
    return q;
}

// Physical flux F(U) . n
template <class T>
__device__ __forceinline__ void euler_flux(const Prim<T>& q, const T* n, T* F) {
    F[0] = q.r * q.un;
#pragma unroll
    for (int a = 0; a < 3; ++a) F[1 + a] = q.r * q.u[a] * q.un + q.p * n[a];
    F[4] = (q.E + q.p) * q.un;
}

// Rusanov: s = max(|u_nL| + c_L, |u_nR| + c_R).
template <class T>
__device__ void rusanov_flux(const Prim<T>& L, const Prim<T>& R, const T* UL, const T* UR, const T* n, T* F) {
    T FL[5], FR[5];
    euler_flux(L, n, FL);
    euler_flux(R, n, FR);
    const T s = fmax(fabs(L.un) + L.c, fabs(R.un) + R.c);
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] = T(0.5) * (FL[v] + FR[v]) - T(0.5) * s * (UR[v] - UL[v]);
}

// HLLC (Toro, Spruce & Speares) with Davis wave speeds; S* >= 0 takes the
// left star state.
template <class T>
__device__ void hllc_flux(const Prim<T>& L, const Prim<T>& R, const T* UL, const T* UR, const T* n, T* F) {
    const T SL = fmin(L.un - L.c, R.un - R.c), SR = fmax(L.un + L.c, R.un + R.c);
    if (SL >= T(0)) {
        euler_flux(L, n, F);
        return;
    }
    if (SR <= T(0)) {
        euler_flux(R, n, F);
        return;
    }
    const T Ss = fdiv(R.p - L.p + L.r * L.un * (SL - L.un) - R.r * R.un * (SR - R.un),
                      L.r * (SL - L.un) - R.r * (SR - R.un));
    const bool left = Ss >= T(0);
    const Prim<T>& K = left ? L : R;
    const T* UK = left ? UL : UR;
    const T SK = left ? SL : SR;
    euler_flux(K, n, F);
    const T rchi = fdiv(K.r * (SK - K.un), SK - Ss);
    T Us[5];
    Us[0] = rchi;
#pragma unroll
    for (int a = 0; a < 3; ++a) Us[1 + a] = rchi * (K.u[a] + (Ss - K.un) * n[a]);
    Us[4] = rchi * (K.E * K.ir + (Ss - K.un) * (Ss + fdiv(K.p, K.r * (SK - K.un))));
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] += SK * (Us[v] - UK[v]);
}

template <class T>
__device__ __forceinline__ void prim_W(const PhysT<T>& P, const T* u, T* W) {
    const T ir = T(1) / u[0];
    W[0] = u[1] * ir;
    W[1] = u[2] * ir;
    W[2] = u[3] * ir;
    W[3] = P.gM2 * pressure(P, u) * ir;
}

// Kind of a boundary tag, selected with compile-time indices (a run-time
// index into the by-value table would move it to scratch memory).
template <class T>
__device__ __forceinline__ int bc_kind(const BcT<T>& B, int tag) {
    int kind = UCNS_BC_TRANSMISSIVE;
#pragma unroll
    for (int t = 1; t < 8; ++t)
        if (t == tag) kind = B.kind[t];
    return kind;
}

// Ghost state across a boundary face: Dirichlet takes the prescribed state,
// the no-slip wall mirrors the velocity of the interior point state `in`,
// the symmetry plane reflects its momentum in the face plane (n the unit
// face normal; either orientation), transmissive outflow copies the interior
// cell average `avg` (zeroth-order extrapolation; copying the reconstructed
// point value would feed the boundary cell's one-sided extrapolation back
// into it).
template <class T>
__device__ __forceinline__ void ghost(const BcT<T>& B, int tag, const T* in, const T* avg, const T* n, T* out) {
    int kind = UCNS_BC_TRANSMISSIVE;
    T st[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int t = 1; t < 8; ++t)
        if (t == tag) {
            kind = B.kind[t];
#pragma unroll
            for (int v = 0; v < 5; ++v) st[v] = B.state[t][v];
        }
    if (kind == UCNS_BC_DIRICHLET) {
#pragma unroll
        for (int v = 0; v < 5; ++v) out[v] = st[v];
    } else if (kind == UCNS_BC_WALL) {
        out[0] = in[0];
        out[1] = -in[1];
        out[2] = -in[2];
        out[3] = -in[3];
        out[4] = in[4];
    } else if (kind == UCNS_BC_SYMMETRY) {
        const T mn2 = T(2) * (in[1] * n[0] + in[2] * n[1] + in[3] * n[2]);
        out[0] = in[0];
#pragma unroll
        for (int a = 0; a < 3; ++a) out[1 + a] = in[1 + a] - mn2 * n[a];
        out[4] = in[4];
    } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) out[v] = avg[v];
    }
}

// ---------------------------------------------------------------- gradients

template <class T>
struct GradArgs {
    const double* U;
    int64_t nc;
    const int32_t* c2f;
    int NF;
    const int32_t* fcell;
    const T* fnrm;
    const T* farea;
    const double* vol;
    const T* glsq;  // [nfmax][3][nc] least-squares weights per face slot
    T* gradW;
};

// Green-Gauss (LSQ false): grad W_i = (1/|V_i|) sum_f (W_i + W_j)/2 n_f |S_f|
// (outward).  Least squares (LSQ true): grad W_i = sum_slots G_slot (W_j - W_i)
// with the fit's weights built with the mesh; boundary slots take the ghost.
template <class T, bool LSQ>
__global__ __launch_bounds__(kBlock) void gradients_kernel(GradArgs<T> A, PhysT<T> P, BcT<T> B) {
    const int64_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= A.nc) return;
    const int64_t nc = A.nc;
    T ui[5], Wi[4], g[12];
#pragma unroll
    for (int v = 0; v < 5; ++v) ui[v] = T(A.U[v * nc + c]);
    prim_W(P, ui, Wi);
#pragma unroll
    for (int k = 0; k < 12; ++k) g[k] = T(0);
    // faces in groups of G: the group's ids, then its geometry and
    // neighbours, then the neighbours' states (three memory waits per group
    // instead of three per face; FP64 takes two groups to stay at 3 waves)
    constexpr int G = sizeof(T) == 4 ? kMaxFaces : kMaxFaces / 2;
#pragma unroll
    for (int g0 = 0; g0 < kMaxFaces; g0 += G) {
        int32_t f2[G], other[G];
#pragma unroll
        for (int i = 0; i < G; ++i) f2[i] = g0 + i < A.NF ? A.c2f[int64_t(g0 + i) * nc + c] : -1;
        // absent slots read face 0 and boundary sides cell 0, and are
        // skipped or replaced below: every load is unconditional (a load
        // under a lane condition would be a branch that waits for it)
        T sa[G], nr[G][3];
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const int64_t f = f2[i] >= 0 ? f2[i] >> 1 : 0;
            const int side = f2[i] & 1;
            other[i] = A.fcell[2 * f + (1 - side)];
            if constexpr (LSQ) {
                // a slot beyond the cell's faces holds zero weights
                const int slot = g0 + i < A.NF ? g0 + i : 0;
                sa[i] = T(0);
#pragma unroll
                for (int a = 0; a < 3; ++a) nr[i][a] = A.glsq[int64_t(3 * slot + a) * nc + c];
            } else {
                sa[i] = (side ? T(-0.5) : T(0.5)) * A.farea[f];
#pragma unroll
                for (int a = 0; a < 3; ++a) nr[i][a] = A.fnrm[3 * f + a];
            }
        }
        T uo[G][5];
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const int64_t j = other[i] >= 0 ? other[i] : 0;
#pragma unroll
            for (int v = 0; v < 5; ++v) uo[i][v] = T(A.U[v * nc + j]);
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
            if (f2[i] < 0) continue;
            if (other[i] < 0) {
                // the symmetry ghost needs the face normal, which the
                // least-squares weights do not carry (boundary faces only)
                T nb[3];
                const int64_t fb = f2[i] >> 1;
#pragma unroll
                for (int a = 0; a < 3; ++a) nb[a] = LSQ ? A.fnrm[3 * fb + a] : nr[i][a];
                ghost(B, -1 - other[i], ui, ui, nb, uo[i]);
            }
            T Wo[4];
            prim_W(P, uo[i], Wo);
#pragma unroll
            for (int var = 0; var < 4; ++var) {
                const T wf = LSQ ? Wo[var] - Wi[var] : (Wi[var] + Wo[var]) * sa[i];
#pragma unroll
                for (int a = 0; a < 3; ++a) g[3 * var + a] += wf * nr[i][a];
            }
        }
    }
    const T iv = LSQ ? T(1) : T(1.0 / A.vol[c]);
#pragma unroll
    for (int k = 0; k < 12; ++k) A.gradW[k * nc + c] = g[k] * iv;
}

// The ghost state of ghost() for the cell-average interior state, the
// boundary table read from device memory with the lane's own tag (a table
// passed by value, selected with compile-time indices, would hold 48 scalar
// registers through the long reconstruction kernels and spill them).
template <class T>
__device__ __forceinline__ void ghost_dev(const ucns_bc* bc, int tag, const T* in, const T* n, T* out) {
    const int t = tag > 0 && tag < 8 ? tag : 0;
    int kind = UCNS_BC_TRANSMISSIVE;
    T st[5] = {T(0), T(0), T(0), T(0), T(0)};
    if (bc && t > 0) {
        kind = bc->kind[t];
#pragma unroll
        for (int v = 0; v < 5; ++v) st[v] = T(bc->state[t][v]);
    }
    // selects, not branches (a branch per kind lets the compiler merge the
    // table loads with the copies of the interior state and move that state
    // to memory); a transmissive slot subtracts an exact zero
    const bool dir = kind == UCNS_BC_DIRICHLET, wall = kind == UCNS_BC_WALL;
    const T mn2 = kind == UCNS_BC_SYMMETRY ? T(2) * (in[1] * n[0] + in[2] * n[1] + in[3] * n[2]) : T(0);
    out[0] = dir ? st[0] : in[0];
#pragma unroll
    for (int a = 0; a < 3; ++a) out[1 + a] = dir ? st[1 + a] : (wall ? -in[1 + a] : in[1 + a] - mn2 * n[a]);
    out[4] = dir ? st[4] : in[4];
}

// Gradient of W of one cell at the end of its reconstruction, the sums of
// gradients_kernel: Green-Gauss (LSQ false) sum_slots (W_i + W_j) w_slot with
// each slot's outward n |S| / (2 |V|) stored with the mesh, or least squares
// (LSQ true) sum_slots (W_j - W_i) G_slot with the fit's weights.  A
// boundary slot's neighbour entry is its face's negative tag (the ghost state
// enters), an absent slot's weights are zero.  The neighbours' states were
// gathered by the cell's central stencil a moment earlier.
template <class T, bool LSQ>
__device__ void cell_gradient(const ReconArgs<T>& A, int64_t c, const double* ui) {
    const int64_t nc = A.nc;
    // W of a state, as prim_W forms it
    auto primw = [&](const T* q, T* W) {
        const T ir = T(1) / q[0];
        W[0] = q[1] * ir;
        W[1] = q[2] * ir;
        W[2] = q[3] * ir;
        W[3] = A.gM2 * (A.gm1 * (q[4] - T(0.5) * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0])) * ir;
    };
    T u[5], Wi[4], g[12];
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = T(ui[v]);
    primw(u, Wi);
#pragma unroll
    for (int k = 0; k < 12; ++k) g[k] = T(0);
    // every load unconditional (a slot beyond the mesh's NF reads slot 0 and
    // is then taken as absent: transmissive ghost, zero weights)
    int32_t jn[kMaxFaces];
    T w[kMaxFaces][3];
#pragma unroll
    for (int lf = 0; lf < kMaxFaces; ++lf) {
        const bool have = lf < A.NF;
        const int64_t r = have ? lf : 0;
        const int32_t j = A.nbr[r * nc + c];
        jn[lf] = have ? j : -1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const T x = (LSQ ? A.glsq : A.ggw)[(3 * r + a) * nc + c];
            w[lf][a] = have ? x : T(0);
        }
    }
    T uo[kMaxFaces][5];
#pragma unroll
    for (int lf = 0; lf < kMaxFaces; ++lf) {
        const int64_t j = jn[lf] >= 0 ? jn[lf] : c;  // boundary slots replaced below
#pragma unroll
        for (int v = 0; v < 5; ++v) uo[lf][v] = T(A.U[v * nc + j]);
    }
#pragma unroll
    for (int lf = 0; lf < kMaxFaces; ++lf) {
        if (jn[lf] < 0) {
            // the symmetry ghost needs the unit normal (either orientation):
            // the direction of the slot's Green-Gauss weight (boundary lanes
            // only read it for the least-squares sum)
            T gw[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) gw[a] = LSQ ? (lf < A.NF ? A.ggw[int64_t(3 * lf + a) * nc + c] : T(0)) : w[lf][a];
            const T wn = sqrt(gw[0] * gw[0] + gw[1] * gw[1] + gw[2] * gw[2]);
            const T iw = wn > T(0) ? T(1) / wn : T(0);
            const T nb[3] = {gw[0] * iw, gw[1] * iw, gw[2] * iw};
            ghost_dev(A.bcd, -1 - jn[lf], u, nb, uo[lf]);
        }
        T Wo[4];
        primw(uo[lf], Wo);
#pragma unroll
        for (int var = 0; var < 4; ++var) {
            const T s2 = LSQ ? Wo[var] - Wi[var] : Wi[var] + Wo[var];
#pragma unroll
            for (int a = 0; a < 3; ++a) g[3 * var + a] += s2 * w[lf][a];
        }
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) A.gradW[k * nc + c] = g[k];
}

// ---------------------------------------------------------------- face flux

template <class T>
struct FluxArgs {
    const double* U;  // cell averages (transmissive ghost)
    const T* fs;
    int64_t nf, nc;
    int Q;
    const int32_t* fcell;
    const uint8_t* flf;  // local face index of each side
    const T* fnrm;
    const T* farea;
    const T* fw;
    const T* fdc;
    const uint8_t* fnq;
    const T* gradW;
    T* ff;
};

// Viscous flux F_v . n with the penalised interface gradient
// grad W_f = (grad W_L + grad W_R)/2 + (4/3)/L_int (W_R - W_L) (x) n on
// W = (u, v, w, T); G0 is the face's mean cell gradient, pen = (4/3)/L_int.
// The stress and heat flux are linear in grad W_f, so they split into the
// face's constant part from G0 (formed once per face) and the penalty part,
// which for the rank-one dW (x) n with |n| = 1 reduces to
//   tau_pen n = mu pen (dW_u + (1/3)(dW_u . n) n),   q_pen = kappa pen dW_T.
template <class T>
struct ViscFace {
    T t0[3], q0;  // mu (G0 + G0^T - (2/3) div G0 I) n and kappa G0_T . n
    T mp, kp;     // mu pen, kappa pen
};

template <class T>
__device__ __forceinline__ ViscFace<T> viscous_face(const PhysT<T>& P, const T* G0, const T* n, T pen) {
    ViscFace<T> V;
    const T div = G0[0] + G0[4] + G0[8];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        T t = T(0);
#pragma unroll
        for (int j = 0; j < 3; ++j) t += (G0[3 * i + j] + G0[3 * j + i]) * n[j];
        V.t0[i] = P.mu * (t - T(2.0 / 3.0) * div * n[i]);
    }
    V.q0 = P.kappa * (G0[9] * n[0] + G0[10] * n[1] + G0[11] * n[2]);
    V.mp = P.mu * pen;
    V.kp = P.kappa * pen;
    return V;
}

// F_v . n at one Gauss point (the work term with the mean velocity).
template <class T>
__device__ __forceinline__ void viscous_flux(const PhysT<T>& P, const ViscFace<T>& V, const Prim<T>& L,
                                             const Prim<T>& R, const T* n, T* Fv) {
    T dW[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) dW[a] = R.u[a] - L.u[a];
    const T dT = P.gM2 * (R.p * R.ir - L.p * L.ir);
    const T dn3 = T(1.0 / 3.0) * (dW[0] * n[0] + dW[1] * n[1] + dW[2] * n[2]);
    T e = V.q0 + V.kp * dT;
    Fv[0] = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const T t = V.t0[i] + V.mp * (dW[i] + dn3 * n[i]);
        Fv[1 + i] = t;
        e += T(0.5) * (L.u[i] + R.u[i]) * t;
    }
    Fv[4] = e;
}

// Face gradient on a symmetry plane: the mean of the cell's gradient and its
// mirror image.  With velocity gradient G (G_ij = du_i/dx_j) and mirror
// M = I - 2 n n^T, (G + M G M)/2 = G - n (n^T G) - (G n) n^T + 2 (n^T G n) n n^T
// (the normal-tangential couplings vanish: no shear stress on the plane);
// the temperature gradient loses its normal part (no heat flux).
template <class T>
__device__ __forceinline__ void symmetry_gradient(T* G, const T* n) {
    T a[3], b[3], s = T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        a[j] = n[0] * G[j] + n[1] * G[3 + j] + n[2] * G[6 + j];
        b[j] = G[3 * j] * n[0] + G[3 * j + 1] * n[1] + G[3 * j + 2] * n[2];
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) s += n[j] * b[j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) G[3 * i + j] += -n[i] * a[j] - b[i] * n[j] + T(2) * s * n[i] * n[j];
    const T gn = G[9] * n[0] + G[10] * n[1] + G[11] * n[2];
#pragma unroll
    for (int j = 0; j < 3; ++j) G[9 + j] -= gn * n[j];
}

// One lane per face; the Gauss-point sum is the lane's own loop.  Adjacent
// lanes take adjacent faces (numbered by owner), so each point-state load of
// a wave reads a few contiguous runs of the owners' and neighbours' slots,
// and the cell gradients and face geometry are read once per face.
template <class T>
__global__ __launch_bounds__(kBlock) void face_flux_kernel(FluxArgs<T> A, PhysT<T> P, BcT<T> B) {
    const int64_t f = xcd_block() * blockDim.x + threadIdx.x;
    if (f >= A.nf) return;
    const int64_t nc = A.nc;
    const int Q = A.Q;
    const int nq = A.fnq[f];
    const T n[3] = {A.fnrm[3 * f], A.fnrm[3 * f + 1], A.fnrm[3 * f + 2]};
    const int32_t cL = A.fcell[2 * f], cR = A.fcell[2 * f + 1];
    // point states in the slot rows [lf][q][cell][v] of each side
    // both sides' local face indices in one 16-bit load (the right one is
    // needed only off the boundary, and a load under that lane condition
    // would wait)
    const uint32_t lf2 = *reinterpret_cast<const uint16_t*>(A.flf + 2 * f);
    const int lfL = int(lf2 & 0xffu), lfR = int(lf2 >> 8);
    const int64_t slot = 5 * fs_cells_padded(nc);  // values per point slot
    const T* pL = A.fs + int64_t(lfL) * Q * slot + int64_t(cL) * 5;
    const T* pR = cR >= 0 ? A.fs + int64_t(lfR) * Q * slot + int64_t(cR) * 5 : pL;
    T avg[5];
    if (cR < 0) {
#pragma unroll
        for (int v = 0; v < 5; ++v) avg[v] = T(A.U[v * nc + cL]);
    }
    T G0[12], pen = T(0);
    ViscFace<T> VF{};
    if (P.viscous) {
        // a boundary face takes its own cell's gradient on both sides; both
        // loads are unconditional (a load under a lane condition would wait)
        const int64_t cRg = cR >= 0 ? cR : cL;
#pragma unroll
        for (int k = 0; k < 12; ++k) G0[k] = T(0.5) * (A.gradW[k * nc + cL] + A.gradW[k * nc + cRg]);
        const T dx = A.fdc[3 * f], dy = A.fdc[3 * f + 1], dz = A.fdc[3 * f + 2];
        pen = T(4.0 / 3.0) / sqrt(dx * dx + dy * dy + dz * dz);
        if (cR < 0 && bc_kind(B, -1 - cR) == UCNS_BC_SYMMETRY) symmetry_gradient(G0, n);
        VF = viscous_face(P, G0, n, pen);
    }
    T F[5] = {T(0), T(0), T(0), T(0), T(0)};
    // FP32 loads the next point's two states while it evaluates this one's
    // flux (FP64 has no registers to spare: 158, three waves per SIMD)
    constexpr bool kAhead = sizeof(T) == 4;
    // (on a boundary face pR = pL and the ghost replaces uR)
    auto load_point = [&](int q, T* uL, T* uR) {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            uL[v] = pL[int64_t(q) * slot + v];
            uR[v] = pR[int64_t(q) * slot + v];
        }
    };
    T uLn[5], uRn[5];
    if (kAhead && nq > 0) load_point(0, uLn, uRn);
#pragma unroll 1  // unrolling doubles the live registers (FP64: 3 waves per SIMD instead of 2)
    for (int q = 0; q < nq; ++q) {
        T uL[5], uR[5], Fq[5];
        if constexpr (kAhead) {
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                uL[v] = uLn[v];
                uR[v] = uRn[v];
            }
            if (q + 1 < nq) load_point(q + 1, uLn, uRn);
        } else {
            load_point(q, uL, uR);
        }
        if (cR < 0) ghost(B, -1 - cR, uL, avg, n, uR);
        const Prim<T> qL = prim(P, uL, n), qR = prim(P, uR, n);
        if (P.flux == UCNS_HLLC)
            hllc_flux(qL, qR, uL, uR, n, Fq);
        else
            rusanov_flux(qL, qR, uL, uR, n, Fq);
        if (P.viscous) {
            T Fv[5];
            viscous_flux(P, VF, qL, qR, n, Fv);
#pragma unroll
            for (int v = 0; v < 5; ++v) Fq[v] -= Fv[v];
        }
        const T w = A.fw[f * Q + q];
#pragma unroll
        for (int v = 0; v < 5; ++v) F[v] += w * Fq[v];
    }
    const T ar = A.farea[f];
#pragma unroll
    for (int v = 0; v < 5; ++v) A.ff[f * 5 + v] = ar * F[v];
}

// ----------------------------------------------------- residual + RK stage

template <class T>
struct ResArgs {
    const T* ff;
    int64_t nc;
    const int32_t* c2f;
    int NF;
    const double* vol;
    double* R;   // residual output (residual only)
    double* U0;  // RK: written at stage 0, read at stages 1 and 2
    double* U;
    const double* dt;
    double a, b;
    int stage;
    // with FINAL: per-block time-step and kinetic-energy partials of the new U
    const double* hdt;
    PhysT<double> P;
    double* part;  // [2][gridDim]
};

// Fixed-shape block reduction (deterministic for a fixed launch shape).
template <bool MIN>
__device__ double block_reduce(double x) {
    __shared__ double sh[kBlock];
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = MIN ? fmin(sh[threadIdx.x], sh[threadIdx.x + s]) : sh[threadIdx.x] + sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

// sum_f s_if F_f over the cell's faces in local order; all face ids first,
// then all face fluxes (two memory waits instead of two per face).
template <class T>
__device__ __forceinline__ void face_sum(const ResArgs<T>& A, int64_t c, double acc[5]) {
    int32_t f2[kMaxFaces];
#pragma unroll
    for (int lf = 0; lf < kMaxFaces; ++lf) f2[lf] = lf < A.NF ? A.c2f[int64_t(lf) * A.nc + c] : -1;
    // absent slots load face 0 and are skipped below (a load under a lane
    // condition would be a branch that waits for it)
    T fl[kMaxFaces][5];
#pragma unroll
    for (int lf = 0; lf < kMaxFaces; ++lf)
#pragma unroll
        for (int v = 0; v < 5; ++v) fl[lf][v] = A.ff[int64_t(f2[lf] >= 0 ? f2[lf] >> 1 : 0) * 5 + v];
#pragma unroll
    for (int v = 0; v < 5; ++v) acc[v] = 0.0;
#pragma unroll
    for (int lf = 0; lf < kMaxFaces; ++lf) {
        if (f2[lf] < 0) continue;
        const double s = (f2[lf] & 1) ? -1.0 : 1.0;
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] += s * double(fl[lf][v]);
    }
}

// Shu-Osher stage update a U0 + b (U + dt R), one explicit rounding order
// for every kernel that applies it.
__device__ __forceinline__ double rk_combine(double a, double b, double u0, double u, double dt, double r) {
    return fma(a, u0, b * fma(dt, r, u));
}

// Admissible time step of one cell (reading of compute_time_step, Listing 1 in
// Sec. 3.2; cfl applied by the caller): h / (|u| + c), and with viscosity
// rho h^2 / (2 mu max(4/3, gamma/Pr)).
// NaN or a non-positive value returns -inf, which poisons the minimum.
__device__ __forceinline__ double cell_dt(const PhysT<double>& P, const double* u, double h) {
    const double sp = sqrt(u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0];
    const double cs = sqrt(P.gamma * pressure(P, u) / u[0]);
    const double ti = h / (sp + cs);  // NaN for a NaN state or a negative pressure
    double t = ti;
    // (fmin would return the viscous bound past a NaN convective one)
    if (P.viscous) t = fmin(t, u[0] * h * h / (2.0 * P.mu * fmax(4.0 / 3.0, P.gamma / P.pr)));
    return ti > 0.0 && t > 0.0 ? t : -INFINITY;
}

// R_i = -(1/|V_i|) sum_f s_if F_f over the cell's faces in local order.
// FINAL (last RK stage): also the block's minimum time step and kinetic-energy
// sum of the new state, into part[blk] and part[nblocks + blk].
template <class T, bool RK, bool FINAL = false>
__global__ __launch_bounds__(kBlock) void residual_kernel(ResArgs<T> A) {
    const int64_t blk = xcd_block();
    const int64_t c = blk * blockDim.x + threadIdx.x;
    if constexpr (FINAL) {
        double tdt = INFINITY, tke = 0.0;
        if (c < A.nc) {
            double acc[5];
            face_sum<T>(A, c, acc);
            const double vol = A.vol[c];
            const double iv = -1.0 / vol;
            const double dt = *A.dt;
            double un[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const int64_t i = v * A.nc + c;
                un[v] = rk_combine(A.a, A.b, A.U0[i], A.U[i], dt, acc[v] * iv);
                A.U[i] = un[v];
            }
            tdt = cell_dt(A.P, un, A.hdt[c]);
            tke = vol * 0.5 * (un[1] * un[1] + un[2] * un[2] + un[3] * un[3]) / un[0];
        }
        const double rdt = block_reduce<true>(tdt);
        const double rke = block_reduce<false>(tke);
        if (threadIdx.x == 0) {
            A.part[blk] = rdt;
            A.part[gridDim.x + blk] = rke;
        }
        return;
    }
    if (c >= A.nc) return;
    double acc[5];
    face_sum<T>(A, c, acc);
    const double iv = -1.0 / A.vol[c];
    if (RK) {
        const double dt = *A.dt;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const int64_t i = v * A.nc + c;
            const double u = A.U[i];
            if (A.stage == 0) {
                A.U0[i] = u;
                A.U[i] = fma(dt, acc[v] * iv, u);
            } else {
                A.U[i] = rk_combine(A.a, A.b, A.U0[i], u, dt, acc[v] * iv);
            }
        }
    } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) A.R[v * A.nc + c] = acc[v] * iv;
    }
}

// Five-stage fourth-order SSP-RK (Spiteri & Ruuth), Shu-Osher form, stage s
// on R = -(1/|V|) sum_f s_f F_f of the current U:
//   s0: u1 = u0 + b10 dt R(u0)                      (W0 <- u0)
//   s1: u2 = a20 u0 + a21 u1 + b21 dt R(u1)         (W1 <- u2)
//   s2: u3 = a30 u0 + a32 u2 + b32 dt R(u2)         (W2 <- u3)
//   s3: u4 = a40 u0 + a43 u3 + b43 dt R(u3)         (W3 <- R(u3))
//   s4: u5 = a52 u2 + a53 u3 + b53 dt R(u3) + a54 u4 + b54 dt R(u4)
struct Ssp54 {
    double b10, a20, a21, b21, a30, a32, b32, a40, a43, b43, a52, a53, b53, a54, b54;
};
constexpr Ssp54 kSsp54{0.391752226571890, 0.444370493651235, 0.555629506348765, 0.368410593050371,
                       0.620101851488403, 0.379898148511597, 0.251891774271694, 0.178079954393132,
                       0.821920045606868, 0.544974750228521, 0.517231671970585, 0.096059710526147,
                       0.063692468666290, 0.386708617503269, 0.226007483236906};

template <class T>
__global__ __launch_bounds__(kBlock) void residual_ssp54_kernel(ResArgs<T> A, double* W) {
    const int64_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= A.nc) return;
    double acc[5];
    face_sum<T>(A, c, acc);
    const double iv = -1.0 / A.vol[c];
    const double dt = *A.dt;
    const int64_t n = 5 * A.nc;
    constexpr Ssp54 k = kSsp54;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        const int64_t i = v * A.nc + c;
        const double u = A.U[i], r = acc[v] * iv;
        double un;
        switch (A.stage) {
            case 0: W[i] = u; un = u + k.b10 * dt * r; break;
            case 1: un = k.a20 * W[i] + k.a21 * u + k.b21 * dt * r; W[n + i] = un; break;
            case 2: un = k.a30 * W[i] + k.a32 * u + k.b32 * dt * r; W[2 * n + i] = un; break;
            case 3: W[3 * n + i] = r; un = k.a40 * W[i] + k.a43 * u + k.b43 * dt * r; break;
            default:
                un = k.a52 * W[n + i] + k.a53 * W[2 * n + i] + k.b53 * dt * W[3 * n + i] + k.a54 * u + k.b54 * dt * r;
                break;
        }
        A.U[i] = un;
    }
}

__global__ __launch_bounds__(kBlock) void rk_stage_kernel(int64_t n, double* U0, const double* R, double* U,
                                                          const double* dt, double a, double b, int stage) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double u = U[i];
    if (stage == 0) {
        U0[i] = u;
        U[i] = fma(*dt, R[i], u);
    } else {
        U[i] = rk_combine(a, b, U0[i], u, *dt, R[i]);
    }
}

// ----------------------------------------------------------------- reductions

__global__ __launch_bounds__(kBlock) void dt_partial_kernel(int64_t nc, const double* U, const double* hdt,
                                                            PhysT<double> P, double* part) {
    double best = INFINITY;
    for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < nc; c += int64_t(gridDim.x) * blockDim.x) {
        double u[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) u[v] = U[v * nc + c];
        best = fmin(best, cell_dt(P, u, hdt[c]));
    }
    const double r = block_reduce<true>(best);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ __launch_bounds__(kBlock) void dt_final_kernel(int nb, const double* part, double cfl, double* dt) {
    double best = INFINITY;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) best = fmin(best, part[i]);
    const double r = block_reduce<true>(best);
    if (threadIdx.x == 0) *dt = (r > 0.0 && r < INFINITY) ? cfl * r : NAN;
}

__global__ __launch_bounds__(kBlock) void ke_partial_kernel(int64_t nc, const double* U, const double* vol, double* part) {
    double s = 0.0;
    for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < nc; c += int64_t(gridDim.x) * blockDim.x) {
        const double r = U[c], mx = U[nc + c], my = U[2 * nc + c], mz = U[3 * nc + c];
        s += vol[c] * 0.5 * (mx * mx + my * my + mz * mz) / r;
    }
    const double t = block_reduce<false>(s);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// dt_final and ke_final of the fused last stage in one launch.
__global__ __launch_bounds__(kBlock) void rk_final_kernel(int nb, const double* part, double cfl, double inv_vol,
                                                          double* dt, double* ke) {
    double best = INFINITY, sum = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        best = fmin(best, part[i]);
        sum += part[nb + i];
    }
    const double r = block_reduce<true>(best);
    const double t = block_reduce<false>(sum);
    if (threadIdx.x == 0) {
        *dt = (r > 0.0 && r < INFINITY) ? cfl * r : NAN;
        *ke = t * inv_vol;
    }
}

__global__ __launch_bounds__(kBlock) void ke_final_kernel(int nb, const double* part, double inv_vol, double* out) {
    // fixed order: each thread sums a strided slice, then a fixed tree
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
    const double t = block_reduce<false>(s);
    if (threadIdx.x == 0) *out = t * inv_vol;
}

// Solenoidal and dilatational dissipation (TGV diagnostics): per-block sums
// of |V| |curl u|^2 and |V| (div u)^2 from the cell velocity gradients
// (gradW rows 3 var + dir), then a fixed-order final sum.
template <class T>
__global__ __launch_bounds__(kBlock) void diss_partial_kernel(int64_t nc, const T* __restrict__ g,
                                                              const double* __restrict__ vol, double* part) {
    double ss = 0.0, sd = 0.0;
    for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < nc; c += int64_t(gridDim.x) * blockDim.x) {
        auto G = [&](int var, int a) { return double(g[(3 * var + a) * nc + c]); };
        const double wx = G(2, 1) - G(1, 2), wy = G(0, 2) - G(2, 0), wz = G(1, 0) - G(0, 1);
        const double dv = G(0, 0) + G(1, 1) + G(2, 2);
        ss += vol[c] * (wx * wx + wy * wy + wz * wz);
        sd += vol[c] * dv * dv;
    }
    const double ts = block_reduce<false>(ss);
    const double td = block_reduce<false>(sd);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = ts;
        part[gridDim.x + blockIdx.x] = td;
    }
}

__global__ __launch_bounds__(kBlock) void diss_final_kernel(int nb, const double* part, double mu_over_vol,
                                                            double* out) {
    double ss = 0.0, sd = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        ss += part[i];
        sd += part[nb + i];
    }
    const double ts = block_reduce<false>(ss);
    const double td = block_reduce<false>(sd);
    if (threadIdx.x == 0) {
        out[0] = mu_over_vol * ts;
        out[1] = 4.0 / 3.0 * mu_over_vol * td;
    }
}

// ----------------------------------------------------------------- helpers

inline unsigned grid_for(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

int hip_check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return UCNS_EHIP;
    }
    return UCNS_OK;
}

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255) == 0; }

#define UCNS_REQUIRE(cond, code, msg) \
    do {                              \
        if (!(cond)) {                \
            set_error(msg);           \
            return code;              \
        }                             \
    } while (0)

template <class T>
const T* arena_ptr(const Arena& a, size_t off) {
    return reinterpret_cast<const T*>(static_cast<const unsigned char*>(a.dev) + off);
}

template <class T>
ReconArgs<T> make_recon_args(const Mesh& m, const Arena& ar, double gm1, const double* U, const ucns_gate* gate,
                             void* fs, uint8_t* flags, float* label, void* gradW = nullptr,
                             const ucns_phys* phys = nullptr, const ucns_bc* bc_device = nullptr) {
    ReconArgs<T> A;
    A.U = U;
    A.nc = m.nc;
    A.sten_c = arena_ptr<int32_t>(ar, ar.sten_c);
    A.Bc = arena_ptr<T>(ar, ar.Bc);
    A.MC = m.mc_pad;
    A.MCmin = m.mc_min;
    A.ndir = arena_ptr<uint8_t>(ar, ar.ndir);
    A.sten_d = arena_ptr<int32_t>(ar, ar.sten_d);
    A.Bd = arena_ptr<T>(ar, ar.Bd);
    A.ND = std::max(1, m.nd_max);
    A.MD = std::max(1, m.md_pad);
    A.O = arena_ptr<T>(ar, ar.O);
    A.xi = arena_ptr<T>(ar, ar.xi);
    A.pmean = arena_ptr<T>(ar, ar.pmean);
    A.cnq = arena_ptr<uint8_t>(ar, ar.cnq);
    A.Q = m.qmax;
    A.NF = m.nfmax;
    A.gate = gate ? gate->mask : nullptr;
    A.mlp = gate ? static_cast<const unsigned char*>(gate->mlp_image) : nullptr;
    A.mask_out = gate ? gate->mask_out : nullptr;
    A.nbr = arena_ptr<int32_t>(ar, ar.nbr);
    A.ndc = arena_ptr<T>(ar, ar.ndc);
    A.hb = arena_ptr<T>(ar, ar.hb);
    A.ncen = arena_ptr<uint8_t>(ar, ar.ncen);
    // the arena's one scratch region (written by the P4 reconstruction call)
    A.ustage = ar.ustage ? reinterpret_cast<double*>(static_cast<unsigned char*>(ar.dev) + ar.ustage) : nullptr;
    A.fs = static_cast<T*>(fs);
    A.flags = flags;
    A.label = label;
    A.lam_c = T(m.lambda_c);
    A.eps = T(m.eps);
    A.gm1 = T(gm1);
    A.gradW = static_cast<T*>(gradW);
    A.ggw = arena_ptr<T>(ar, ar.ggw);
    A.glsq = arena_ptr<T>(ar, ar.glsq);
    A.bcd = bc_device;
    A.gM2 = phys ? T(phys->gamma * phys->mach * phys->mach) : T(0);
    return A;
}

// Cell gradients of W = (u, v, w, T) in a pass of their own.
template <class T>
void launch_gradients(const Mesh& m, const Arena& ar, const ucns_phys* phys, const ucns_bc* bc, const double* U,
                      void* gradW, hipStream_t st) {
    GradArgs<T> A{U, m.nc, arena_ptr<int32_t>(ar, ar.c2f), m.nfmax, arena_ptr<int32_t>(ar, ar.fcell),
                  arena_ptr<T>(ar, ar.fnrm), arena_ptr<T>(ar, ar.farea), arena_ptr<double>(ar, ar.vol),
                  arena_ptr<T>(ar, ar.glsq), static_cast<T*>(gradW)};
    if (phys->grad == UCNS_GRAD_LSQ)
        hipLaunchKernelGGL((gradients_kernel<T, true>), dim3(grid_for(m.nc)), dim3(kBlock), 0, st, A,
                           make_phys<T>(phys), make_bc<T>(bc));
    else
        hipLaunchKernelGGL((gradients_kernel<T, false>), dim3(grid_for(m.nc)), dim3(kBlock), 0, st, A,
                           make_phys<T>(phys), make_bc<T>(bc));
}

template <class T, int K>
int launch_recon_k(const ReconArgs<T>& A, hipStream_t st, bool grad_lsq = false) {
    if (A.Q > face_qmax<K>()) return UCNS_EINVAL;
    if (recon_span_bytes(A.nc, int(sizeof(T)), K, A.NF) > kMaxDescriptorBytes) return UCNS_EINVAL;
    const dim3 grid(grid_for(A.nc)), block(kBlock);
    if (A.gradW) {
        // the fused gradients (grad_lsq: least squares, else Green-Gauss): P2
        // only (the P3 kernels have no scalar registers to spare for the
        // extra arguments)
        if constexpr (K == 9) {
            if (A.label) return UCNS_EINVAL;
            const bool gate = A.mlp || A.gate;
            if (grad_lsq && gate)
                hipLaunchKernelGGL((reconstruct_kernel<T, K, false, true, 2>), grid, block, 0, st, A);
            else if (grad_lsq)
                hipLaunchKernelGGL((reconstruct_kernel<T, K, false, false, 2>), grid, block, 0, st, A);
            else if (gate)
                hipLaunchKernelGGL((reconstruct_kernel<T, K, false, true, 1>), grid, block, 0, st, A);
            else
                hipLaunchKernelGGL((reconstruct_kernel<T, K, false, false, 1>), grid, block, 0, st, A);
        } else {
            return UCNS_EINVAL;
        }
    } else if (A.mlp || A.gate) {
        hipLaunchKernelGGL((reconstruct_kernel<T, K, false, true>), grid, block, 0, st, A);
    } else {
        if (A.label)
            hipLaunchKernelGGL((reconstruct_kernel<T, K, true, false>), grid, block, 0, st, A);
        else
            hipLaunchKernelGGL((reconstruct_kernel<T, K, false, false>), grid, block, 0, st, A);
    }
    hipLaunchKernelGGL((reconstruct_fallback_kernel<T, K>), grid, block, 0, st, A);
    return UCNS_OK;
}

// P4: one lane per (cell, variable), 12 cells per wave; full CWENOZ only
// (the gate's network is trained on P2 features).
template <class T>
int launch_recon_p4(const ReconArgs<T>& A, hipStream_t st) {
    if (A.Q > kP4Q || A.NF > kMaxFaces || A.mlp || A.gate || !A.ustage) return UCNS_EINVAL;
    if (recon_span_bytes(A.nc, int(sizeof(T)), kP4K, A.NF) > kMaxDescriptorBytes) return UCNS_EINVAL;
    hipLaunchKernelGGL(p4_stage_state_kernel, dim3(grid_for(A.nc)), dim3(kBlock), 0, st, A.U, A.nc, A.ustage);
    const int64_t per_block = int64_t(kBlock / 64) * kP4Cells;
    const dim3 grid(unsigned((A.nc + per_block - 1) / per_block)), block(kBlock);
    if (A.label)
        hipLaunchKernelGGL((reconstruct_p4_kernel<T, true>), grid, block, 0, st, A);
    else
        hipLaunchKernelGGL((reconstruct_p4_kernel<T, false>), grid, block, 0, st, A);
    hipLaunchKernelGGL((reconstruct_p4_fallback_kernel<T>), dim3(grid_for(A.nc)), block, 0, st, A);
    return UCNS_OK;
}

// gradW (optional, P2): the gradients of U by phys->grad as well, formed by
// the reconstruction kernel at the end of each cell.
template <class T>
int launch_recon(const Mesh& m, const Arena& ar, double gm1, const double* U, const ucns_gate* gate, void* fs,
                 uint8_t* flags, float* label, hipStream_t st, void* gradW = nullptr, const ucns_phys* phys = nullptr,
                 const ucns_bc* bc_device = nullptr) {
    const ReconArgs<T> A = make_recon_args<T>(m, ar, gm1, U, gate, fs, flags, label, gradW, phys, bc_device);
    const bool lsq = phys && phys->grad == UCNS_GRAD_LSQ;
    if (m.K == 9) return launch_recon_k<T, 9>(A, st, lsq);
    if (m.K == 19) return launch_recon_k<T, 19>(A, st, lsq);
    if (m.K == kP4K && !gradW) return launch_recon_p4<T>(A, st);
    return UCNS_EINVAL;
}

template <class T>
int launch_features(const Mesh& m, const Arena& ar, const double* U, float* out, hipStream_t st) {
    if (recon_span_bytes(m.nc, int(sizeof(T)), m.K, m.nfmax) > kMaxDescriptorBytes) return UCNS_EINVAL;
    const ReconArgs<T> A = make_recon_args<T>(m, ar, 0.4, U, nullptr, nullptr, nullptr, nullptr);
    if (m.K == 9)
        hipLaunchKernelGGL((gate_features_kernel<T, 9>), dim3(grid_for(m.nc)), dim3(kBlock), 0, st, A, out);
    else if (m.K == 19)
        hipLaunchKernelGGL((gate_features_kernel<T, 19>), dim3(grid_for(m.nc)), dim3(kBlock), 0, st, A, out);
    else
        return UCNS_EINVAL;
    return UCNS_OK;
}

}  // namespace

// ============================================ static scratch (no allocation)

// Per-block reduction partials of ucns_residual_rk_final_noalloc: a fixed
// device array (4 MiB on every GPU the library runs on, held until the
// process ends), so that call allocates nothing.  Its host-side name is not
// a device address: each device's copy is looked up once with
// hipGetSymbolAddress and only that pointer is used.
constexpr int64_t kStaticScratchBlocks = int64_t(1) << 18;
static __device__ __align__(256) double scratch[2 * kStaticScratchBlocks];

// Per-block gradient partials of ucns_mlp_train_step (1.3 MiB per GPU), in
// the same kind of fixed array: training steps on one GPU run in stream order.
static __device__ __align__(256) float train_part[mlp::kTrainMaxBlocks * mlp::kTrainStride];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
void* g_train_part_ptr[kMaxDevices] = {};

// Device address of a file-scope device array on the current device, looked
// up once per device and kept in table.
int symbol_address(const void* symbol, void** table, const char* name, void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
        return UCNS_EHIP;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index beyond the static scratch table");
        return UCNS_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!table[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, symbol);
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress(") + name + "): " + hipGetErrorString(e));
            return UCNS_EHIP;
        }
        table[dev] = p;
    }
    *out = table[dev];
    return UCNS_OK;
}

int static_scratch(double** out) {
    void* p = nullptr;
    const int rc = symbol_address(HIP_SYMBOL(scratch), g_scratch_ptr, "scratch", &p);
    *out = static_cast<double*>(p);
    return rc;
}
}  // namespace

// =================================================================== C ABI

struct ucns_mesh_impl_guard {};

extern "C" {

const char* ucns_last_error(void) { return ucns::last_error_cstr(); }

int ucns_mesh_build(const ucns_mesh_desc* desc, const ucns_recon_opts* opts, int n_threads, ucns_mesh** out) {
    UCNS_REQUIRE(out != nullptr, UCNS_EINVAL, "null output handle");
    *out = nullptr;
    Mesh* m = nullptr;
    int rc = build_mesh(desc, opts, n_threads, &m);
    if (rc != UCNS_OK) return rc;
    *out = new ucns_mesh{m};
    return UCNS_OK;
}

void ucns_mesh_free(ucns_mesh* mesh) {
    if (!mesh) return;
    delete mesh->m;
    delete mesh;
}

int ucns_mesh_info(const ucns_mesh* mesh, int64_t* info) {
    UCNS_REQUIRE(mesh && info, UCNS_EINVAL, "null argument");
    const Mesh& m = *mesh->m;
    int64_t v[16] = {m.nc, m.nf, m.K, m.qmax, m.nfmax, m.mc_pad, m.nd_max, m.md_pad, m.nbnd, m.n_dropped_total,
                     m.mc_min, m.mc_pad, m.order, m.kd, 0, 0};
    std::memcpy(info, v, sizeof v);
    return UCNS_OK;
}

int ucns_mesh_arena_bytes(const ucns_mesh* mesh, int precision, size_t* bytes) {
    UCNS_REQUIRE(mesh && bytes, UCNS_EINVAL, "null argument");
    UCNS_REQUIRE(precision == UCNS_F64 || precision == UCNS_F32, UCNS_EINVAL, "bad precision");
    Arena a;
    pack_arena(*mesh->m, precision, a, nullptr);
    *bytes = a.bytes;
    return UCNS_OK;
}

int ucns_recon_span_bytes(int64_t n_cell, int precision, int n_unknowns, int n_face_slots, uint64_t* span) {
    UCNS_REQUIRE(span && n_cell >= 0 && n_unknowns > 0 && n_face_slots > 0, UCNS_EINVAL, "bad argument");
    UCNS_REQUIRE(precision == UCNS_F64 || precision == UCNS_F32, UCNS_EINVAL, "bad precision");
    *span = recon_span_bytes(n_cell, precision == UCNS_F64 ? 8 : 4, n_unknowns, n_face_slots);
    return UCNS_OK;
}

int ucns_mesh_upload(ucns_mesh* mesh, int precision, void* arena, size_t bytes, ucns_stream stream) {
    UCNS_REQUIRE(mesh && arena, UCNS_EINVAL, "null argument");
    UCNS_REQUIRE(precision == UCNS_F64 || precision == UCNS_F32, UCNS_EINVAL, "bad precision");
    UCNS_REQUIRE(aligned(arena), UCNS_EINVAL, "arena must be 256-byte aligned");
    Mesh& m = *mesh->m;
    Arena a;
    std::vector<unsigned char> image;
    pack_arena(m, precision, a, &image);
    UCNS_REQUIRE(bytes >= a.bytes, UCNS_ENOMEM, "arena smaller than ucns_mesh_arena_bytes");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(arena, image.data(), a.bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_error(std::string("upload: ") + hipGetErrorString(e));
        return UCNS_EHIP;
    }
    a.dev = arena;
    m.arena[precision] = a;
    return UCNS_OK;
}

int ucns_mesh_release(ucns_mesh* mesh, int precision) {
    UCNS_REQUIRE(mesh, UCNS_EINVAL, "null argument");
    UCNS_REQUIRE(precision == UCNS_F64 || precision == UCNS_F32, UCNS_EINVAL, "bad precision");
    mesh->m->arena[precision].dev = nullptr;
    return UCNS_OK;
}

int ucns_mesh_faces(const ucns_mesh* mesh, int32_t* c2f, int64_t* fcell, double* qp, double* shift) {
    UCNS_REQUIRE(mesh, UCNS_EINVAL, "null argument");
    const Mesh& m = *mesh->m;
    if (c2f) std::memcpy(c2f, m.c2f.data(), sizeof(int32_t) * m.c2f.size());
    if (fcell) std::memcpy(fcell, m.fcell.data(), sizeof(int64_t) * m.fcell.size());
    if (qp) std::memcpy(qp, m.fqp.data(), sizeof(double) * m.fqp.size());
    if (shift) std::memcpy(shift, m.fshift.data(), sizeof(double) * m.fshift.size());
    return UCNS_OK;
}

int ucns_mesh_cell_geometry(const ucns_mesh* mesh, double* vol, double* cen, double* hbasis) {
    UCNS_REQUIRE(mesh, UCNS_EINVAL, "null argument");
    const Mesh& m = *mesh->m;
    if (vol) std::memcpy(vol, m.vol.data(), sizeof(double) * m.nc);
    if (cen) std::memcpy(cen, m.cen.data(), sizeof(double) * 3 * m.nc);
    if (hbasis) std::memcpy(hbasis, m.hb.data(), sizeof(double) * m.nc);
    return UCNS_OK;
}

int ucns_mesh_stencil(const ucns_mesh* mesh, int64_t cell, int64_t* central, int32_t* ncen, int64_t* dir,
                      int32_t* ndir, int32_t* dface) {
    UCNS_REQUIRE(mesh && central && ncen && dir && ndir && dface, UCNS_EINVAL, "null argument");
    const Mesh& m = *mesh->m;
    UCNS_REQUIRE(cell >= 0 && cell < m.nc, UCNS_EINVAL, "cell out of range");
    *ncen = m.ncen[cell];
    for (int k = 0; k < m.ncen[cell]; ++k) central[k] = m.cand[size_t(cell) * kMaxCentral + k];
    for (int s = 0; s < m.ndir[cell]; ++s) {
        ndir[s] = m.nds[cell * kMaxFaces + s];
        dface[s] = m.dface[cell * kMaxFaces + s];
        for (int k = 0; k < ndir[s]; ++k) dir[s * kMaxDir + k] = m.dir[(size_t(cell) * kMaxFaces + s) * kMaxDir + k];
    }
    return m.ndir[cell];
}

int ucns_mesh_operators(const ucns_mesh* mesh, int64_t cell, double* Bc, double* Bd, double* O, double* Phi) {
    UCNS_REQUIRE(mesh, UCNS_EINVAL, "null argument");
    const Mesh& m = *mesh->m;
    UCNS_REQUIRE(cell >= 0 && cell < m.nc, UCNS_EINVAL, "cell out of range");
    const int K = m.K;
    if (Bc)
        for (int k = 0; k < K; ++k)
            for (int j = 0; j < m.ncen[cell]; ++j) Bc[k * m.ncen[cell] + j] = m.Bc[(size_t(cell) * K + k) * m.mc_pad + j];
    if (Bd)
        for (int s = 0; s < m.ndir[cell]; ++s)
            for (int k = 0; k < m.kd; ++k)
                for (int j = 0; j < m.nds[cell * kMaxFaces + s]; ++j)
                    Bd[(s * m.kd + k) * kMaxDir + j] = m.Bd[((size_t(cell) * m.nd_max + s) * m.kd + k) * m.md_pad + j];
    if (O) std::memcpy(O, &m.O[size_t(cell) * K * K], sizeof(double) * K * K);
    if (Phi) std::memcpy(Phi, &m.Phi[size_t(cell) * m.nfmax * m.qmax * K], sizeof(double) * m.nfmax * m.qmax * K);
    return UCNS_OK;
}

int ucns_mesh_gradient_weights(const ucns_mesh* mesh, int64_t cell, double* G) {
    UCNS_REQUIRE(mesh && G, UCNS_EINVAL, "null argument");
    const Mesh& m = *mesh->m;
    UCNS_REQUIRE(cell >= 0 && cell < m.nc, UCNS_EINVAL, "cell out of range");
    std::memcpy(G, &m.glsq[size_t(cell) * kMaxFaces * 3], sizeof(double) * kMaxFaces * 3);
    return UCNS_OK;
}

int ucns_workspace_elems(const ucns_mesh* mesh, int64_t* face_state, int64_t* face_flux, int64_t* gradW,
                         int64_t* reduce_scratch) {
    UCNS_REQUIRE(mesh, UCNS_EINVAL, "null argument");
    const Mesh& m = *mesh->m;
    if (face_state) *face_state = int64_t(m.nfmax) * m.qmax * 5 * fs_cells_padded(m.nc);
    if (face_flux) *face_flux = m.nf * 5;
    if (gradW) *gradW = 12 * m.nc;
    if (reduce_scratch) *reduce_scratch = std::max<int64_t>(kRedBlocks, 2 * int64_t(grid_for(m.nc)));
    return UCNS_OK;
}

int ucns_dt(const ucns_mesh* mesh, const ucns_phys* phys, const double* U, double cfl, double* scratch,
            double* dt_dev, ucns_stream stream) {
    UCNS_REQUIRE(mesh && phys && U && scratch && dt_dev, UCNS_EINVAL, "null argument");
    const Mesh& m = *mesh->m;
    const Arena& a = m.arena[UCNS_F64].dev ? m.arena[UCNS_F64] : m.arena[UCNS_F32];
    UCNS_REQUIRE(a.dev, UCNS_ESTATE, "mesh not uploaded");
    UCNS_REQUIRE(cfl > 0, UCNS_EINVAL, "cfl must be positive");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    PhysT<double> P = make_phys<double>(phys);
    unsigned nb = std::min<unsigned>(kRedBlocks, grid_for(m.nc));
    hipLaunchKernelGGL(dt_partial_kernel, dim3(nb), dim3(kBlock), 0, st, m.nc, U, arena_ptr<double>(a, a.hdt), P, scratch);
    hipLaunchKernelGGL(dt_final_kernel, dim3(1), dim3(kBlock), 0, st, int(nb), scratch, cfl, dt_dev);
    return hip_check("ucns_dt");
}

namespace {
int reconstruct_impl(const ucns_mesh* mesh, const ucns_phys* phys, const ucns_bc* bc_device, const double* U,
                     int precision,
                     const ucns_gate* gate, void* face_state, uint8_t* flags, float* label, void* gradW,
                     ucns_stream stream, const char* name) {
    UCNS_REQUIRE(mesh && phys && U && face_state && flags, UCNS_EINVAL, "null argument");
    UCNS_REQUIRE(precision == UCNS_F64 || precision == UCNS_F32, UCNS_EINVAL, "bad precision");
    UCNS_REQUIRE(aligned(U) && aligned(face_state), UCNS_EINVAL, "device buffers must be 256-byte aligned");
    const Mesh& m = *mesh->m;
    const Arena& ar = m.arena[precision];
    UCNS_REQUIRE(ar.dev, UCNS_ESTATE, "mesh not uploaded for this precision");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    UCNS_REQUIRE(!(gate && gate->mask && gate->mlp_image), UCNS_EINVAL, "gate: give a mask or a network, not both");
    UCNS_REQUIRE(!(gate && gate->mlp_image) || aligned(gate->mlp_image), UCNS_EINVAL,
                 "gate: the network image must be 256-byte aligned");
    UCNS_REQUIRE(!(gate && (gate->mask || gate->mlp_image) && label), UCNS_EINVAL,
                 "labels are produced by the ungated reconstruction only");

    const double gm1 = phys->gamma - 1.0;
    const int rc = precision == UCNS_F64
                       ? launch_recon<double>(m, ar, gm1, U, gate, face_state, flags, label, st, gradW, phys, bc_device)
                       : launch_recon<float>(m, ar, gm1, U, gate, face_state, flags, label, st, gradW, phys, bc_device);
    if (rc != UCNS_OK) {
        set_error("unsupported reconstruction order or face-point count, a gate at P4 (its network is trained "
                  "at P2), or a mesh beyond the 4 GiB span of one buffer descriptor (ucns_recon_span_bytes)");
        return rc;
    }
    return hip_check(name);
}
}  // namespace

int ucns_reconstruct(const ucns_mesh* mesh, const ucns_phys* phys, const double* U, int precision,
                     const ucns_gate* gate, void* face_state, uint8_t* flags, float* label, ucns_stream stream) {
    return reconstruct_impl(mesh, phys, nullptr, U, precision, gate, face_state, flags, label, nullptr, stream,
                            "ucns_reconstruct");
}

int ucns_reconstruct_gradients(const ucns_mesh* mesh, const ucns_phys* phys, const ucns_bc* bc_device,
                               const double* U, int precision, const ucns_gate* gate, void* face_state,
                               uint8_t* flags, void* gradW, ucns_stream stream) {
    UCNS_REQUIRE(mesh && phys && gradW, UCNS_EINVAL, "null argument");
    UCNS_REQUIRE(phys->grad == UCNS_GRAD_GREEN_GAUSS || phys->grad == UCNS_GRAD_LSQ, UCNS_EINVAL,
                 "bad gradient method");
    UCNS_REQUIRE(mesh->m->order == 2, UCNS_EINVAL, "the fused pass covers order 2; orders 3 and 4: ucns_gradients");
    UCNS_REQUIRE(aligned(gradW), UCNS_EINVAL, "device buffers must be 256-byte aligned");
    return reconstruct_impl(mesh, phys, bc_device, U, precision, gate, face_state, flags, nullptr, gradW, stream,
                            "ucns_reconstruct_gradients");
}

int ucns_gradients(const ucns_mesh* mesh, const ucns_phys* phys, const ucns_bc* bc, const double* U, int precision,
                   void* gradW, ucns_stream stream) {
    UCNS_REQUIRE(mesh && phys && U && gradW, UCNS_EINVAL, "null argument");
    UCNS_REQUIRE(precision == UCNS_F64 || precision == UCNS_F32, UCNS_EINVAL, "bad precision");
    UCNS_REQUIRE(phys->grad == UCNS_GRAD_GREEN_GAUSS || phys->grad == UCNS_GRAD_LSQ, UCNS_EINVAL,
                 "bad gradient method");
    UCNS_REQUIRE(aligned(U) && aligned(gradW), UCNS_EINVAL, "device buffers must be 256-byte aligned");
    const Mesh& m = *mesh->m;
    const Arena& ar = m.arena[precision];
    UCNS_REQUIRE(ar.dev, UCNS_ESTATE, "mesh not uploaded for this precision");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (precision == UCNS_F64)
        launch_gradients<double>(m, ar, phys, bc, U, gradW, st);
    else
        launch_gradients<float>(m, ar, phys, bc, U, gradW, st);
    return hip_check("ucns_gradients");
}

int ucns_face_flux(const ucns_mesh* mesh, const ucns_phys* phys, const ucns_bc* bc, const double* U,
                   const void* face_state, const void* gradW, int precision, void* face_flux, ucns_stream stream) {
    UCNS_REQUIRE(mesh && phys && U && face_state && face_flux, UCNS_EINVAL, "null argument");
    UCNS_REQUIRE(precision == UCNS_F64 || precision == UCNS_F32, UCNS_EINVAL, "bad precision");
    UCNS_REQUIRE(!phys->viscous || gradW, UCNS_EINVAL, "viscous flux needs gradients");
    UCNS_REQUIRE(aligned(face_state) && aligned(face_flux), UCNS_EINVAL, "device buffers must be 256-byte aligned");
    UCNS_REQUIRE(phys->flux == UCNS_HLLC || phys->flux == UCNS_RUSANOV, UCNS_EINVAL, "unknown flux");
    const Mesh& m = *mesh->m;
    const Arena& ar = m.arena[precision];
    UCNS_REQUIRE(ar.dev, UCNS_ESTATE, "mesh not uploaded for this precision");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    auto go = [&](auto zero) {
        using T = decltype(zero);
        FluxArgs<T> A{U, static_cast<const T*>(face_state), m.nf, m.nc, m.qmax, arena_ptr<int32_t>(ar, ar.fcell),
                      arena_ptr<uint8_t>(ar, ar.flf), arena_ptr<T>(ar, ar.fnrm), arena_ptr<T>(ar, ar.farea), arena_ptr<T>(ar, ar.fw),
                      arena_ptr<T>(ar, ar.fdc), arena_ptr<uint8_t>(ar, ar.fnq), static_cast<const T*>(gradW),
                      static_cast<T*>(face_flux)};
        hipLaunchKernelGGL((face_flux_kernel<T>), dim3(grid_for(m.nf)), dim3(kBlock), 0, st, A, make_phys<T>(phys),
                           make_bc<T>(bc));
    };
    if (precision == UCNS_F64)
        go(double(0));
    else
        go(float(0));
    return hip_check("ucns_face_flux");
}

namespace {
int launch_residual(const ucns_mesh* mesh, const void* face_flux, int precision, double* R, int stage,
                    const double* dt_dev, double* U0, double* U, ucns_stream stream) {
    static const double Ac[3] = {0.0, 0.75, 1.0 / 3.0}, Bc_[3] = {1.0, 0.25, 2.0 / 3.0};
    const Mesh& m = *mesh->m;
    const Arena& ar = m.arena[precision];
    UCNS_REQUIRE(ar.dev, UCNS_ESTATE, "mesh not uploaded for this precision");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    auto go = [&](auto zero) {
        using T = decltype(zero);
        ResArgs<T> A{static_cast<const T*>(face_flux), m.nc, arena_ptr<int32_t>(ar, ar.c2f), m.nfmax,
                     arena_ptr<double>(ar, ar.vol), R, U0, U, dt_dev, stage >= 0 ? Ac[stage] : 0.0,
                     stage >= 0 ? Bc_[stage] : 0.0, stage};
        if (stage >= 0)
            hipLaunchKernelGGL((residual_kernel<T, true>), dim3(grid_for(m.nc)), dim3(kBlock), 0, st, A);
        else
            hipLaunchKernelGGL((residual_kernel<T, false>), dim3(grid_for(m.nc)), dim3(kBlock), 0, st, A);
    };
    if (precision == UCNS_F64)
        go(double(0));
    else
        go(float(0));
    return hip_check("ucns_residual");
}
}  // namespace

int ucns_residual(const ucns_mesh* mesh, const void* face_flux, int precision, double* R, ucns_stream stream) {
    UCNS_REQUIRE(mesh && face_flux && R, UCNS_EINVAL, "null argument");
    UCNS_REQUIRE(precision == UCNS_F64 || precision == UCNS_F32, UCNS_EINVAL, "bad precision");
    UCNS_REQUIRE(aligned(face_flux) && aligned(R), UCNS_EINVAL, "device buffers must be 256-byte aligned");
    return launch_residual(mesh, face_flux, precision, R, -1, nullptr, nullptr, nullptr, stream);
}

int ucns_residual_rk_stage(const ucns_mesh* mesh, const void* face_flux, int precision, int stage,
                           const double* dt_dev, double* U0, double* U, ucns_stream stream) {
    UCNS_REQUIRE(mesh && face_flux && dt_dev && U0 && U, UCNS_EINVAL, "null argument");
    UCNS_REQUIRE(precision == UCNS_F64 || precision == UCNS_F32, UCNS_EINVAL, "bad precision");
    UCNS_REQUIRE(stage >= 0 && stage <= 2, UCNS_EINVAL, "stage must be 0, 1 or 2");
    UCNS_REQUIRE(aligned(face_flux) && aligned(U0) && aligned(U), UCNS_EINVAL, "device buffers must be 256-byte aligned");
    return launch_residual(mesh, face_flux, precision, nullptr, stage, dt_dev, U0, U, stream);
}

int ucns_residual_ssp54_stage(const ucns_mesh* mesh, const void* face_flux, int precision, int stage,
                              const double* dt_dev, double* W, double* U, ucns_stream stream) {
    UCNS_REQUIRE(mesh && face_flux && dt_dev && W && U, UCNS_EINVAL, "null argument");
    UCNS_REQUIRE(precision == UCNS_F64 || precision == UCNS_F32, UCNS_EINVAL, "bad precision");
    UCNS_REQUIRE(stage >= 0 && stage <= 4, UCNS_EINVAL, "stage must be 0 .. 4");
    UCNS_REQUIRE(aligned(face_flux) && aligned(W) && aligned(U), UCNS_EINVAL, "device buffers must be 256-byte aligned");
    const Mesh& m = *mesh->m;
    const Arena& ar = m.arena[precision];
    UCNS_REQUIRE(ar.dev, UCNS_ESTATE, "mesh not uploaded for this precision");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    auto go = [&](auto zero) {
        using T = decltype(zero);
        ResArgs<T> A{static_cast<const T*>(face_flux), m.nc, arena_ptr<int32_t>(ar, ar.c2f), m.nfmax,
                     arena_ptr<double>(ar, ar.vol), nullptr, nullptr, U, dt_dev, 0.0, 0.0, stage};
        hipLaunchKernelGGL(residual_ssp54_kernel<T>, dim3(grid_for(m.nc)), dim3(kBlock), 0, st, A, W);
    };
    if (precision == UCNS_F64)
        go(double(0));
    else
        go(float(0));
    return hip_check("ucns_residual_ssp54_stage");
}

int ucns_rk_stage(const ucns_mesh* mesh, int stage, const double* dt_dev, double* U0, const double* R,
                  double* U, ucns_stream stream) {
    static const double Ac[3] = {0.0, 0.75, 1.0 / 3.0}, Bc_[3] = {1.0, 0.25, 2.0 / 3.0};
    UCNS_REQUIRE(mesh && dt_dev && U0 && R && U, UCNS_EINVAL, "null argument");
    UCNS_REQUIRE(stage >= 0 && stage <= 2, UCNS_EINVAL, "stage must be 0, 1 or 2");
    UCNS_REQUIRE(aligned(U0) && aligned(R) && aligned(U), UCNS_EINVAL, "device buffers must be 256-byte aligned");
    const int64_t n = 5 * mesh->m->nc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(rk_stage_kernel, dim3(grid_for(n)), dim3(kBlock), 0, st, n, U0, R, U, dt_dev, Ac[stage],
                       Bc_[stage], stage);
    return hip_check("ucns_rk_stage");
}

namespace {
// The last SSP-RK3 stage with the step's reductions; `scratch` holds the
// 2 x grid_for(n_cell) per-block partials (time step, kinetic energy).
int launch_rk_final(const ucns_mesh* mesh, const ucns_phys* phys, const void* face_flux, int precision,
                    const double* dt_dev, double* U0, double* U, double cfl, double* scratch, double* dt_next_dev,
                    double* ke_dev, ucns_stream stream) {
    const Mesh& m = *mesh->m;
    const Arena& ar = m.arena[precision];
    UCNS_REQUIRE(ar.dev, UCNS_ESTATE, "mesh not uploaded for this precision");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const unsigned nb = grid_for(m.nc);
    auto go = [&](auto zero) {
        using T = decltype(zero);
        ResArgs<T> A{static_cast<const T*>(face_flux), m.nc, arena_ptr<int32_t>(ar, ar.c2f), m.nfmax,
                     arena_ptr<double>(ar, ar.vol), nullptr, U0, U, dt_dev, 1.0 / 3.0, 2.0 / 3.0, 2,
                     arena_ptr<double>(ar, ar.hdt), make_phys<double>(phys), scratch};
        hipLaunchKernelGGL((residual_kernel<T, true, true>), dim3(nb), dim3(kBlock), 0, st, A);
    };
    if (precision == UCNS_F64)
        go(double(0));
    else
        go(float(0));
    hipLaunchKernelGGL(rk_final_kernel, dim3(1), dim3(kBlock), 0, st, int(nb), scratch, cfl, 1.0 / m.total_vol,
                       dt_next_dev, ke_dev);
    return hip_check("ucns_residual_rk_final");
}
}  // namespace

int ucns_residual_rk_final(const ucns_mesh* mesh, const ucns_phys* phys, const void* face_flux, int precision,
                           const double* dt_dev, double* U0, double* U, double cfl, double* scratch,
                           double* dt_next_dev, double* ke_dev, ucns_stream stream) {
    UCNS_REQUIRE(mesh && phys && face_flux && dt_dev && U0 && U && scratch && dt_next_dev && ke_dev, UCNS_EINVAL,
                 "null argument");
    UCNS_REQUIRE(precision == UCNS_F64 || precision == UCNS_F32, UCNS_EINVAL, "bad precision");
    UCNS_REQUIRE(cfl > 0, UCNS_EINVAL, "cfl must be positive");
    UCNS_REQUIRE(aligned(face_flux) && aligned(U0) && aligned(U), UCNS_EINVAL, "device buffers must be 256-byte aligned");
    return launch_rk_final(mesh, phys, face_flux, precision, dt_dev, U0, U, cfl, scratch, dt_next_dev, ke_dev, stream);
}

int ucns_residual_rk_final_noalloc(const ucns_mesh* mesh, const ucns_phys* phys, const void* face_flux,
                                   int precision, const double* dt_dev, double* U0, double* U, double cfl,
                                   double* dt_next_dev, double* ke_dev, ucns_stream stream) {
    UCNS_REQUIRE(mesh && phys && face_flux && dt_dev && U0 && U && dt_next_dev && ke_dev, UCNS_EINVAL,
                 "null argument");
    UCNS_REQUIRE(precision == UCNS_F64 || precision == UCNS_F32, UCNS_EINVAL, "bad precision");
    UCNS_REQUIRE(cfl > 0, UCNS_EINVAL, "cfl must be positive");
    UCNS_REQUIRE(aligned(face_flux) && aligned(U0) && aligned(U), UCNS_EINVAL, "device buffers must be 256-byte aligned");
    UCNS_REQUIRE(int64_t(grid_for(mesh->m->nc)) <= kStaticScratchBlocks, UCNS_EINVAL,
                 "ucns_residual_rk_final_noalloc: more than 67,108,864 cells (its static scratch holds the "
                 "partials of 262,144 blocks); use ucns_residual_rk_final with a workspace");
    double* part = nullptr;
    const int rc = static_scratch(&part);
    if (rc != UCNS_OK) return rc;
    return launch_rk_final(mesh, phys, face_flux, precision, dt_dev, U0, U, cfl, part, dt_next_dev, ke_dev, stream);
}

int ucns_diag_ke(const ucns_mesh* mesh, const double* U, double* scratch, double* ke_dev, ucns_stream stream) {
    UCNS_REQUIRE(mesh && U && scratch && ke_dev, UCNS_EINVAL, "null argument");
    const Mesh& m = *mesh->m;
    const Arena& a = m.arena[UCNS_F64].dev ? m.arena[UCNS_F64] : m.arena[UCNS_F32];
    UCNS_REQUIRE(a.dev, UCNS_ESTATE, "mesh not uploaded");
    const double tv = m.total_vol;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    unsigned nb = std::min<unsigned>(kRedBlocks, grid_for(m.nc));
    hipLaunchKernelGGL(ke_partial_kernel, dim3(nb), dim3(kBlock), 0, st, m.nc, U, arena_ptr<double>(a, a.vol), scratch);
    hipLaunchKernelGGL(ke_final_kernel, dim3(1), dim3(kBlock), 0, st, int(nb), scratch, 1.0 / tv, ke_dev);
    return hip_check("ucns_diag_ke");
}

int ucns_diag_dissipation(const ucns_mesh* mesh, const ucns_phys* phys, const void* gradW, int precision,
                          double* scratch, double* eps_dev, ucns_stream stream) {
    UCNS_REQUIRE(mesh && phys && gradW && scratch && eps_dev, UCNS_EINVAL, "null argument");
    UCNS_REQUIRE(precision == UCNS_F64 || precision == UCNS_F32, UCNS_EINVAL, "bad precision");
    UCNS_REQUIRE(phys->reynolds > 0, UCNS_EINVAL, "dissipation needs a Reynolds number");
    const Mesh& m = *mesh->m;
    const Arena& a = m.arena[precision];
    UCNS_REQUIRE(a.dev, UCNS_ESTATE, "mesh not uploaded for this precision");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const unsigned nb = std::min<unsigned>(kRedBlocks, grid_for(m.nc));
    const double* vol = arena_ptr<double>(a, a.vol);
    if (precision == UCNS_F64)
        hipLaunchKernelGGL(diss_partial_kernel<double>, dim3(nb), dim3(kBlock), 0, st, m.nc,
                           static_cast<const double*>(gradW), vol, scratch);
    else
        hipLaunchKernelGGL(diss_partial_kernel<float>, dim3(nb), dim3(kBlock), 0, st, m.nc,
                           static_cast<const float*>(gradW), vol, scratch);
    hipLaunchKernelGGL(diss_final_kernel, dim3(1), dim3(kBlock), 0, st, int(nb), scratch,
                       1.0 / (phys->reynolds * m.total_vol), eps_dev);
    return hip_check("ucns_diag_dissipation");
}

int ucns_check(const double* dt_dev, ucns_stream stream) {
    UCNS_REQUIRE(dt_dev, UCNS_EINVAL, "null argument");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(st);
    double dt = 0.0;
    if (e == hipSuccess) e = hipMemcpy(&dt, dt_dev, sizeof dt, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        set_error(std::string("ucns_check: ") + hipGetErrorString(e));
        return UCNS_EHIP;
    }
    // the reductions write NaN when any cell's time step is NaN or not
    // positive (a NaN or Inf state, negative density or pressure)
    if (!(dt > 0.0 && dt < INFINITY)) {
        set_error("ucns_check: the time step is NaN, infinite or not positive (a cell state is NaN/Inf or has "
                  "non-positive density or pressure)");
        return UCNS_ENUM;
    }
    return UCNS_OK;
}

int ucns_gate_features(const ucns_mesh* mesh, const double* U, int precision, float* features, ucns_stream stream) {
    UCNS_REQUIRE(mesh && U && features, UCNS_EINVAL, "null argument");
    UCNS_REQUIRE(precision == UCNS_F64 || precision == UCNS_F32, UCNS_EINVAL, "bad precision");
    UCNS_REQUIRE(aligned(U) && aligned(features), UCNS_EINVAL, "device buffers must be 256-byte aligned");
    const Mesh& m = *mesh->m;
    const Arena& ar = m.arena[precision];
    UCNS_REQUIRE(ar.dev, UCNS_ESTATE, "mesh not uploaded for this precision");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int rc = precision == UCNS_F64 ? launch_features<double>(m, ar, U, features, st)
                                         : launch_features<float>(m, ar, U, features, st);
    if (rc != UCNS_OK) {
        set_error("unsupported reconstruction order, or a mesh beyond the 4 GiB span of one buffer descriptor "
                  "(ucns_recon_span_bytes)");
        return rc;
    }
    return hip_check("ucns_gate_features");
}

int ucns_mlp_forward(const float* params, const float* features, int64_t n, float* prob, ucns_stream stream) {
    UCNS_REQUIRE(params && features && prob && n >= 0, UCNS_EINVAL, "bad argument");
    if (n == 0) return UCNS_OK;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), params, features, n, prob, nullptr);
    return hip_check("ucns_mlp_forward");
}

int ucns_mlp_pack(const float* params, void* image, ucns_stream stream) {
    UCNS_REQUIRE(params && image, UCNS_EINVAL, "null argument");
    UCNS_REQUIRE(aligned(image), UCNS_EINVAL, "the image must be 256-byte aligned");
    hipLaunchKernelGGL(mlp_pack_kernel, dim3(1), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), params,
                       static_cast<unsigned char*>(image));
    return hip_check("ucns_mlp_pack");
}

int ucns_gate_mask(const float* params, const float* features, int64_t n, uint8_t* mask, ucns_stream stream) {
    UCNS_REQUIRE(params && features && mask && n >= 0, UCNS_EINVAL, "bad argument");
    if (n == 0) return UCNS_OK;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), params, features, n, nullptr, mask);
    return hip_check("ucns_gate_mask");
}

int ucns_mlp_train_step(float* params, float* grads, float* adam_state, const float* features, const float* labels,
                        int64_t n, float pos_weight, float lr, int t, float* loss_dev, ucns_stream stream) {
    UCNS_REQUIRE(params && grads && adam_state && features && labels && n > 0 && t >= 1, UCNS_EINVAL, "bad argument");
    void* p = nullptr;
    const int rc = symbol_address(HIP_SYMBOL(train_part), g_train_part_ptr, "train_part", &p);
    if (rc != UCNS_OK) return rc;
    float* part = static_cast<float*>(p);
    const int nblk = int(std::min<int64_t>((n + 63) / 64, mlp::kTrainMaxBlocks));
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(mlp_train_kernel, dim3(nblk), dim3(64), 0, s, params, part, features, labels, n, pos_weight);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((mlp::kNParam + 256) / 256), dim3(256), 0, s, params, grads, adam_state,
                       adam_state + mlp::kNParam, part, nblk, 1.f / float(n), lr, t, loss_dev);
    return hip_check("ucns_mlp_train_step");
}

}  // extern "C"
