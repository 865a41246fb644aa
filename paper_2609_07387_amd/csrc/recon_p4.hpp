// P4 (CWENOZ5) reconstruction kernel (included by ucns_kernels.hip).
//
// Sec. 2.2 of the UCNS3D v4 paper at fifth order: a central polynomial of
// degree 4 (34 zero-mean basis terms) on the central stencil, one quadratic
// directional polynomial (9 terms) per face on a sectorial stencil, their
// smoothness indicators and WENO-Z weights (eq. cwenoz_weights), the CWENOZ
// blend (eq. cwenoz_poly, Levy-Puppo-Russo form) and the point values at the
// cell's 6 x 16 face Gauss points.
//
// A quad of lanes per cell, 16 cells per wave.  Lane h of the quad owns the
// basis terms g = 4 i + h (i = 0..8; terms 34 and 35 of lanes 2 and 3 are
// padding held at zero) for all five variables: 45 coefficients per lane,
// and every operator row a lane loads is its own (the four lanes of a quad
// read four different rows of the cell's operator, so no value is fetched
// twice).  The lanes' shares of a quadratic form or of a point value meet
// through quad DPP moves; each lane loads two of the five variables of a
// stencil member's state and the quad broadcasts the other three.  Sums over
// the quad are formed as (l0 + l1) + (l2 + l3) in every lane, so all four
// lanes hold the same bits and take the same decisions.

constexpr int kP4K = 34;        // basis terms of the degree-4 polynomial
constexpr int kP4KD = 9;        // basis terms of a quadratic directional polynomial
constexpr int kP4Cells = 16;    // cells per wave
constexpr int kP4Q = 16;        // Gauss points per quadrilateral face (4 x 4)
constexpr int kP4T = 9;         // central terms per lane
constexpr int kP4TD = 3;        // directional terms per lane (g = 4 i + h < 9)
constexpr int kP4NO = kP4K * (kP4K + 1) / 2;  // rows of the upper triangle of O
// Waves per SIMD the kernel is built for (FP64: 256 VGPRs; FP32: 168, a
// few values spilled, measured faster than 2 waves without spills) and how
// many members ahead of the arithmetic the operator rows load.
constexpr int kP4Waves64 = 2, kP4Waves32 = 3;
constexpr int kP4OpAhead64 = 1, kP4OpAhead32 = 1;

// The 34 monomials of degree 1..4 in graded-lex order (x exponent
// descending, then y) at a face point's scaled offset.
template <class T>
__device__ __forceinline__ void monomials_p4(T x, T y, T z, T* t) {
    const T xx = x * x, yy = y * y, zz = z * z;
    const T m[kP4K] = {x, y, z,
                       xx, x * y, x * z, yy, y * z, zz,
                       xx * x, xx * y, xx * z, x * yy, x * y * z, x * zz, yy * y, yy * z, y * zz, zz * z,
                       xx * xx, xx * x * y, xx * x * z, xx * yy, xx * y * z, xx * zz, x * yy * y, x * yy * z,
                       x * y * zz, x * zz * z, yy * yy, yy * y * z, yy * zz, y * zz * z, zz * zz};
#pragma unroll
    for (int k = 0; k < kP4K; ++k) t[k] = m[k];
}

// Quad DPP move: lane l of each group of four reads lane sel_l of the same
// group; CTRL is the quad_perm control (two bits per destination lane).
template <int CTRL>
__device__ __forceinline__ int quad_mov(int x) {
    return __builtin_amdgcn_mov_dpp(x, CTRL, 0xf, 0xf, false);
}
template <int CTRL, class T>
__device__ __forceinline__ T quad_mov(T x) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, quad_mov<CTRL>(__builtin_bit_cast(int, x)));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, x);
        const uint32_t lo = uint32_t(quad_mov<CTRL>(int(uint32_t(u))));
        const uint32_t hi = uint32_t(quad_mov<CTRL>(int(uint32_t(u >> 32))));
        return __builtin_bit_cast(T, (uint64_t(hi) << 32) | lo);
    }
}
constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E, kQuadXor3 = 0x1B;  // [1,0,3,2] [2,3,0,1] [3,2,1,0]
constexpr int kQuadLane0 = 0x00, kQuadLane1 = 0x55, kQuadLane2 = 0xAA, kQuadLane3 = 0xFF;

template <int X, class T>
__device__ __forceinline__ T quad_xor(T x) {
    if constexpr (X == 1)
        return quad_mov<kQuadXor1>(x);
    else if constexpr (X == 2)
        return quad_mov<kQuadXor2>(x);
    else
        return quad_mov<kQuadXor3>(x);
}

// (l0 + l1) + (l2 + l3) in every lane of the quad (the same bits everywhere:
// each addition is commutative)
template <class T>
__device__ __forceinline__ T quad_sum(T x) {
    const T p = x + quad_xor<1>(x);
    return p + quad_xor<2>(p);
}

// Row of O (upper triangle, row-major) of the term pair (p, q), p <= q;
// rows past the last (padding terms) are clamped into the array.
__device__ __forceinline__ int p4_tri(int p, int q) {
    const int r = p * kP4K - (p * (p - 1)) / 2 + (q - p);
    return r < kP4NO ? r : kP4NO - 1;
}

// Jumps of a stencil member's five variables, U_m - U_c in FP64 rounded to
// T: lane k of the quad loaded variable k (broadcast to the quad), every
// lane loaded variable 4.
template <class T>
__device__ __forceinline__ void p4_jumps(double uh, double u4, const double* ui, T* bv) {
    bv[0] = T(quad_mov<kQuadLane0>(uh) - ui[0]);
    bv[1] = T(quad_mov<kQuadLane1>(uh) - ui[1]);
    bv[2] = T(quad_mov<kQuadLane2>(uh) - ui[2]);
    bv[3] = T(quad_mov<kQuadLane3>(uh) - ui[3]);
    bv[4] = T(u4 - ui[4]);
}

// The member stream of a list of stencils: member q (q = 0 .. n-1) has its
// id at row q of `sten` and its KR operator rows at rows q KR .. of `op`
// (each [row][cell]); the lane loads the rows at its byte offsets off[].
// body(q, bv, b) receives the member's five jumps and the lane's operator
// values.  Loads run ahead of the arithmetic in 8-member trips with
// compile-time register slots (no register is copied while its load is in
// flight, and the DPP moves keep the compiler from unrolling a runtime loop
// itself):
//  ids: one load per 4 members, lane h of the quad taking member 4g + h
//       (broadcast to the quad when used), 5 to 8 members ahead;
//  states: 3 members ahead (4 slots of 2 values);
//  operators: DB members ahead (DB + 1 slots, DB + 1 divides 8).
// Rows past the last member read the last one, so every step issues the
// same loads.
template <class T, int NTL, int DB, class Body>
__device__ __forceinline__ void p4_stream(const int32_t* sten, const T* op, int KR, int n, int64_t nc, uint32_t c4,
                                          const uint32_t* off, __amdgpu_buffer_rsrc_t rS, uint32_t hofs,
                                          const double* ui, int h, Body&& body) {
    constexpr int RB = DB + 1;
    static_assert(8 % RB == 0, "operator slots must divide the trip");
    const uint32_t rowI = uint32_t(nc) * 4u;
    auto group = [&](int g) {
        const int r0 = min(4 * g, n - 1);
        const int o = min(4 * g + h, n - 1) - r0;
        return bld<int32_t>(row_rsrc(sten, r0, nc, 4), c4 + uint32_t(o) * rowI, 0u);
    };
    auto load_b = [&](int q, T* b) {
        const auto rB = row_rsrc(op, int64_t(min(q, n - 1)) * KR, nc, KR);
#pragma unroll
        for (int i = 0; i < NTL; ++i) b[i] = bld<T>(rB, off[i], 0u);
    };
    auto load_u = [&](int32_t j, double& uh, double& u4) {  // from the staged [cell][8] state
        uh = bld<double>(rS, uint32_t(j) * 64u + hofs, 0u);
        u4 = bld<double>(rS, uint32_t(j) * 64u + 32u, 0u);
    };
    int32_t gA = group(0), gB = group(1);  // members 0..3 and 4..7
    double uh[4], u4[4];
    T b[RB][NTL];
    load_u(quad_mov<kQuadLane0>(gA), uh[0], u4[0]);
    load_u(quad_mov<kQuadLane1>(gA), uh[1], u4[1]);
    load_u(quad_mov<kQuadLane2>(gA), uh[2], u4[2]);
#pragma unroll
    for (int d = 0; d < DB; ++d) load_b(d, b[d]);
#pragma unroll 1
    for (int q0 = 0; q0 < n; q0 += 8) {
        static_for<0, 8>([&](auto S) {
            constexpr int s = decltype(S)::value;
            constexpr int L = (s + 3) % 4, CTRL = 0x55 * L;
            const int q = q0 + s;
            // member q + 3: slot A's lane 3 at s = 0, slot B's lanes at
            // s = 1..4, the next A group's lanes 0..2 at s = 5..7
            const int32_t j = quad_mov<CTRL>((s == 0 || s >= 5) ? gA : gB);
            load_u(j, uh[(s + 3) % 4], u4[(s + 3) % 4]);
            if constexpr (s == 0) gA = group(q0 / 4 + 2);  // members q0 + 8 .. q0 + 11
            if constexpr (s == 4) gB = group(q0 / 4 + 3);  // members q0 + 12 .. q0 + 15
            load_b(q + DB, b[(s + DB) % RB]);
            if (q < n) {  // uniform
                T bv[5];
                p4_jumps<T>(uh[s % 4], u4[s % 4], ui, bv);
                body(q, bv, b[s % RB]);
            }
        });
    }
}

// One lane's share of the quadratic forms a_v^T O a_v (v = 0..4) over the
// lane's NT terms g_i = 4 i + h, with tbase[i] the row of the pair (g_i, g_i):
//  own pairs (i <= j): weight 1 on the diagonal, 2 off it, row
//  tbase[i] + 4 (j - i);
//  with lane h ^ X (partner term g'_j = 4 j + (h ^ X)): pairs i < j with
//  weight 2 (g_i < g'_j, row tbase[i] + 4 (j - i) + (h ^ X) - h) and the
//  diagonal pairs i = j with weight 2 in the lower lane of the two only.
//  Summed over the quad every ordered pair of distinct terms counts once and
//  each term's square once.
template <class T, int NT>
__device__ __forceinline__ void p4_form_own(const T* __restrict__ O, int64_t nc, int64_t c, const int* tbase,
                                            const T (*a)[NT], T* s) {
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        T t[5];
        const T od = O[int64_t(tbase[i]) * nc + c];
#pragma unroll
        for (int v = 0; v < 5; ++v) t[v] = od * a[v][i];
#pragma unroll
        for (int j = i + 1; j < NT; ++j) {
            const T o = T(2) * O[int64_t(min(tbase[i] + 4 * (j - i), kP4NO - 1)) * nc + c];
#pragma unroll
            for (int v = 0; v < 5; ++v) t[v] += o * a[v][j];
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) s[v] += a[v][i] * t[v];
    }
}

template <int X, class T, int NT>
__device__ __forceinline__ void p4_form_cross(const T* __restrict__ O, int64_t nc, int64_t c, int h, const int* tbase,
                                              const T (*a)[NT], T* s) {
    const int dh = (h ^ X) - h;
    const T wdiag = dh > 0 ? T(2) : T(0);
    const int ddiag = dh > 0 ? dh : 0;  // the upper lane reads a valid row it weights by zero
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        T ap[5];  // the partner's coefficients of its term j
#pragma unroll
        for (int v = 0; v < 5; ++v) ap[v] = quad_xor<X>(a[v][j]);
        T t[5];
        {
            const T o = wdiag * O[int64_t(min(tbase[j] + ddiag, kP4NO - 1)) * nc + c];
#pragma unroll
            for (int v = 0; v < 5; ++v) t[v] = o * a[v][j];
        }
#pragma unroll
        for (int i = 0; i < j; ++i) {
            const T o = T(2) * O[int64_t(min(tbase[i] + 4 * (j - i) + dh, kP4NO - 1)) * nc + c];
#pragma unroll
            for (int v = 0; v < 5; ++v) t[v] += o * a[v][i];
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) s[v] += ap[v] * t[v];
    }
}

// a_v^T O a_v for the five variables, complete in every lane of the quad
// (a sum of squares: a rounded value below zero is clamped).
template <class T, int NT>
__device__ __forceinline__ void p4_forms(const T* __restrict__ O, int64_t nc, int64_t c, int h, const int* tbase,
                                         const T (*a)[NT], T* out) {
    T s[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) s[v] = T(0);
    p4_form_own<T, NT>(O, nc, c, tbase, a, s);
    p4_form_cross<1, T, NT>(O, nc, c, h, tbase, a, s);
    p4_form_cross<2, T, NT>(O, nc, c, h, tbase, a, s);
    p4_form_cross<3, T, NT>(O, nc, c, h, tbase, a, s);
#pragma unroll
    for (int v = 0; v < 5; ++v) out[v] = fmax(quad_sum(s[v]), T(0));
}

// The state staged cell-interleaved, [cell][8] doubles (5 used): a stencil
// member's five values then share one 64-byte segment, one cache line for
// the quad where the [5][cell] rows of U would take five.
__global__ __launch_bounds__(kBlock) void p4_stage_state_kernel(const double* __restrict__ U, int64_t nc,
                                                               double* __restrict__ S) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    double v[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] = U[k * nc + c];
    double2* o = reinterpret_cast<double2*>(S + c * 8);
    o[0] = double2{v[0], v[1]};
    o[1] = double2{v[2], v[3]};
    S[c * 8 + 4] = v[4];
}

// Steps per quad (cell c; lane h owns the terms g = 4 i + h of all variables):
//  (i)   jumps b_m = U_m - U_c in FP64, rounded to T
//  (ii)  a = B_c b (34 terms)
//  (iii) SI_1 = a^T O a
//  (iv)  per directional stencil s: a_s = B_s b_s (9 terms), SI_s = a_s^T O_9 a_s
//        with O_9 the block of O on the first 9 (degree <= 2) terms
//  (v)   tau = mean_s |SI_1 - SI_s|; LPR blend
//        abar = s1 a + (tau/W) G on the first 9 terms, s1 = (1 + tau/(eps+SI_1))/W,
//        W = 1 + tau sum_s lambda_s/(eps+SI_s), G = sum_s lambda_s (r_s - r_1) a_s
//  (vi)  point values U_c + Phi_q . abar; positivity of rho and p at each point.
// Every step per variable (component-wise).  LABEL: also the max over
// stencils and variables of |omega - lambda| per cell.
template <class T, bool LABEL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? kP4Waves32 : kP4Waves64)))
void reconstruct_p4_kernel(ReconArgs<T> A) {
    constexpr int K = kP4K, KD = kP4KD, NT = kP4T, NTD = kP4TD;
    const int64_t nc = A.nc;
    const int lane = int(threadIdx.x & 63u);
    const int slot = lane >> 2, h = lane & 3;
    const int64_t c0 = (xcd_block() * (kBlock / 64) + int64_t(threadIdx.x >> 6)) * kP4Cells;
    const bool valid = c0 + slot < nc;
    // quads past the last cell shadow the wave's first cell (every load stays in range)
    const int64_t c = valid ? c0 + slot : (c0 < nc ? c0 : nc - 1);
    double ui[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) ui[v] = A.U[v * nc + c];
    // Stencil streams are buffer loads: the member's rows in a scalar
    // descriptor, the lane's byte offset in a 32-bit register (the launcher
    // bounds every such span below 4 GiB).
    const uint32_t cT = uint32_t(c) * uint32_t(sizeof(T)), c4 = uint32_t(c) * 4u;
    const uint32_t rowT = uint32_t(nc) * uint32_t(sizeof(T));
    const auto rS = rsrc(A.ustage, uint64_t(nc) * 64u);  // the staged [cell][8] state
    const uint32_t hofs = uint32_t(h) * 8u;              // the lane's variable in a cell's record
    // operator rows of the lane's terms (padding terms read the last row),
    // as byte offsets, and their diagonal rows of O
    int trow[NT], tbase[NT];
    uint32_t toff[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        const int g = 4 * i + h < K ? 4 * i + h : K;
        trow[i] = g < K ? g : K - 1;
        tbase[i] = p4_tri(g, g);
        toff[i] = cT + uint32_t(trow[i]) * rowT;
    }

    // (ii) central coefficients; member m's id at sten_c[m][c], its K
    // operator rows at Bc[m][k][c].
    T a[5][NT];
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
        for (int i = 0; i < NT; ++i) a[v][i] = T(0);
    p4_stream<T, NT, sizeof(T) == 4 ? kP4OpAhead32 : kP4OpAhead64>(A.sten_c, A.Bc, K, A.MC, nc, c4, toff, rS, hofs, ui, h,
                                             [&](int, const T* bv, const T* b) {
#pragma unroll
                                                 for (int v = 0; v < 5; ++v)
#pragma unroll
                                                     for (int i = 0; i < NT; ++i) a[v][i] += b[i] * bv[v];
                                             });
    if (4 * (NT - 1) + h >= K) {
#pragma unroll
        for (int v = 0; v < 5; ++v) a[v][NT - 1] = T(0);
    }

    // (iii) SI_1 = a^T O a
    T SI1[5];
    p4_forms<T, NT>(A.O, nc, c, h, tbase, a, SI1);
    // the terms of degree 3 and 4 (i >= 3) take no part in the directional
    // step: parked in LDS (each lane its own slots) until the blend
    __shared__ T park[kBlock / 64][5 * (NT - NTD)][64];
    const int wv = int(threadIdx.x >> 6);
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
        for (int i = NTD; i < NT; ++i) park[wv][v * (NT - NTD) + i - NTD][lane] = a[v][i];

    // (iv) directional stencils: the lane's terms g = 4 i + h < 9 (i < 3)
    const int nd = int(A.ndir[c]);
    const T lam_s = T(1) / (A.lam_c + T(nd > 0 ? nd : 1)), lam_1 = A.lam_c * lam_s;
    T r1[5], G[5][NTD], tsum[5], Lam[5];
    T rs[LABEL ? kMaxFaces : 1][5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        r1[v] = T(1) / (A.eps + SI1[v]);
        tsum[v] = T(0);
        Lam[v] = lam_1 * r1[v];
#pragma unroll
        for (int i = 0; i < NTD; ++i) G[v][i] = T(0);
        if constexpr (LABEL) {
#pragma unroll
            for (int s = 0; s < kMaxFaces; ++s) rs[s][v] = r1[v];
        }
    }
    if (nd > 0) {  // uniform within a quad
        uint32_t doff[NTD];  // the lane's directional operator rows as byte offsets
#pragma unroll
        for (int i = 0; i < NTD; ++i) doff[i] = cT + uint32_t(4 * i + h < KD ? 4 * i + h : KD - 1) * rowT;
        const int MD = A.MD;
#pragma unroll 1
        for (int s = 0; s < A.ND; ++s) {
            T as[5][NTD];
#pragma unroll
            for (int v = 0; v < 5; ++v)
#pragma unroll
                for (int i = 0; i < NTD; ++i) as[v][i] = T(0);
            p4_stream<T, NTD, sizeof(T) == 4 ? kP4OpAhead32 : kP4OpAhead64>(A.sten_d + int64_t(s) * MD * nc, A.Bd + int64_t(s) * MD * KD * nc,
                                                      KD, MD, nc, c4, doff, rS, hofs, ui, h,
                                                      [&](int, const T* bv, const T* b) {
#pragma unroll
                                                          for (int v = 0; v < 5; ++v)
#pragma unroll
                                                              for (int i = 0; i < NTD; ++i) as[v][i] += b[i] * bv[v];
                                                      });
            if (4 * (NTD - 1) + h >= KD) {
#pragma unroll
                for (int v = 0; v < 5; ++v) as[v][NTD - 1] = T(0);
            }
            if (s < nd) {
                // SI_s with the block of O on the first KD terms
                T SIs[5];
                p4_forms<T, NTD>(A.O, nc, c, h, tbase, as, SIs);
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    tsum[v] += fabs(SI1[v] - SIs[v]);
                    const T r = T(1) / (A.eps + SIs[v]);
                    Lam[v] += lam_s * r;
                    if constexpr (LABEL) {
#pragma unroll
                        for (int t = 0; t < kMaxFaces; ++t)
                            if (t == s) rs[t][v] = r;
                    }
                    const T coef = lam_s * (r - r1[v]);
#pragma unroll
                    for (int i = 0; i < NTD; ++i) G[v][i] += coef * as[v][i];
                }
            }
        }
    }
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
        for (int i = NTD; i < NT; ++i) a[v][i] = park[wv][v * (NT - NTD) + i - NTD][lane];
    // (v) blend
    float lab = 0.f;
    if (nd > 0) {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const T tau = tsum[v] / T(nd);
            const T W = T(1) + tau * Lam[v];
            const T s1 = (T(1) + tau * r1[v]) / W;
            const T tw = tau / W;
#pragma unroll
            for (int i = 0; i < NT; ++i) a[v][i] *= s1;
#pragma unroll
            for (int i = 0; i < NTD; ++i)
                if (4 * i + h < KD) a[v][i] += tw * G[v][i];
            if constexpr (LABEL) {
                lab = fmaxf(lab, float(fabs(lam_1 * (s1 - T(1)))));
#pragma unroll
                for (int s = 0; s < kMaxFaces; ++s)
                    if (s < nd) lab = fmaxf(lab, float(fabs(lam_s * ((T(1) + tau * rs[s][v]) / W - T(1)))));
            }
        }
    }

    // (vi) point values at the cell's face points, slot rows [lf][q][cell][v]:
    // lane h writes variable h, lane 0 also variable 4
    T pm[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) pm[i] = A.pmean[int64_t(trow[i]) * nc + c];
    bool ok = true;
    // The face points as one sequence p = lf Q + q, in trips of 8 points.
    // Offsets load four points per instruction (lane h of the quad takes
    // point 4g + h, broadcast to the quad when used) and 5 to 8 points
    // ahead, with the point count of each point's face.
    const int Q = A.Q, NP = A.NF * A.Q;
    auto group = [&](int g, T* xo, int& nq) {
        const int pp = min(4 * g + h, NP - 1);
        const T* X = A.xi + int64_t(pp) * 3 * nc + c;
        xo[0] = X[0];
        xo[1] = X[nc];
        xo[2] = X[2 * nc];
        nq = A.cnq[int64_t(pp / Q) * nc + c];
    };
    auto point = [&](int p, T x, T y, T z) {
        T t[K];
        monomials_p4<T>(x, y, z, t);
        T d[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) d[v] = T(0);
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            // the lane's term 4 i + h (padding terms carry zero coefficients)
            const T t0 = t[4 * i], t1 = t[min(4 * i + 1, K - 1)], t2 = t[min(4 * i + 2, K - 1)],
                    t3 = t[min(4 * i + 3, K - 1)];
            const T ph = (h == 0 ? t0 : h == 1 ? t1 : h == 2 ? t2 : t3) - pm[i];
#pragma unroll
            for (int v = 0; v < 5; ++v) d[v] += ph * a[v][i];
        }
        T val[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) val[v] = T(ui[v] + double(quad_sum(d[v])));
        T* out = A.fs + (int64_t(p) * fs_cells_padded(nc) + c) * 5;
        if (valid) {
            out[h] = h == 0 ? val[0] : h == 1 ? val[1] : h == 2 ? val[2] : val[3];
            if (h == 0) out[4] = val[4];
        }
        const T pr = A.gm1 * (val[4] - T(0.5) * (val[1] * val[1] + val[2] * val[2] + val[3] * val[3]) / val[0]);
        ok = ok && (val[0] > T(1e-10)) && (pr > T(1e-10));
    };
    T xa[3], xb[3];
    int na, nb;
    group(0, xa, na);
    group(1, xb, nb);
#pragma unroll 1
    for (int p0 = 0; p0 < NP; p0 += 8) {
        static_for<0, 8>([&](auto S) {
            constexpr int s = decltype(S)::value, CTRL = 0x55 * (s % 4);
            const int p = p0 + s;
            const T* xg = s < 4 ? xa : xb;
            const T x = quad_mov<CTRL>(xg[0]), y = quad_mov<CTRL>(xg[1]), z = quad_mov<CTRL>(xg[2]);
            const int nq = quad_mov<CTRL>(s < 4 ? na : nb);
            if constexpr (s == 3) group(p0 / 4 + 2, xa, na);  // points p0 + 8 .. p0 + 11
            if constexpr (s == 7) group(p0 / 4 + 3, xb, nb);  // points p0 + 12 .. p0 + 15
            if (p < NP && p - (p / Q) * Q < nq) point(p, x, y, z);  // uniform within a quad
        });
    }
    if (valid && h == 0) {
        A.flags[c] = uint8_t(ok ? 0 : 0x80);
        if constexpr (LABEL) A.label[c] = lab;
    }
}

// Positivity fallback at P4: the main pass is full CWENOZ, so a marked cell
// falls back to first order (its average at every own face point; bit 2).
template <class T>
__global__ __launch_bounds__(kBlock) void reconstruct_p4_fallback_kernel(ReconArgs<T> A) {
    const int64_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= A.nc) return;
    const uint8_t fl = A.flags[c];
    if (!(fl & 0x80)) return;
    const int64_t nc = A.nc;
    for (int lf = 0; lf < A.NF; ++lf) {
        const int nq = A.cnq[int64_t(lf) * nc + c];
        for (int q = 0; q < nq; ++q)
            for (int v = 0; v < 5; ++v)
                A.fs[((int64_t(lf) * A.Q + q) * fs_cells_padded(nc) + c) * 5 + v] = T(A.U[v * nc + c]);
    }
    A.flags[c] = uint8_t((fl & 0x7f) | 4);
}
