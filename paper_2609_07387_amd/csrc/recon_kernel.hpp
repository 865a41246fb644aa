// CWENOZ reconstruction kernel (included by ucns_kernels.hip).
//
// Sec. 2.2 of the UCNS3D v4 paper: least-squares central and directional
// polynomials (eq. lsq_system), smoothness indicators and WENO-Z nonlinear
// weights (eq. cwenoz_weights), the CWENOZ blend (eq. cwenoz_poly) and the
// point values at the cell's face quadrature points.
//
// One thread per cell, all five conserved variables, so every operator value
// is loaded once and used five times.  Every stream of loads (stencil
// members, directional members, face points) is software-pipelined: while
// member i is accumulated, the state and operator values of the next DEPTH
// members and the index of the one after are already in flight, so a wave
// keeps several members' worth of loads outstanding instead of waiting a
// full memory round trip per stencil member.

// Buffer loads: the array's base and size sit in a resource descriptor in
// scalar registers, a small row offset (wave-uniform) in a scalar register
// and the lane's byte offset in one 32-bit vector register, so no access
// needs per-lane 64-bit address arithmetic.  Offsets are 32-bit: a row index
// that can grow with the stencil or face-point count goes into the
// descriptor's 64-bit base instead (row_rsrc), so the only offsets left are a
// few rows of one array, and the launcher refuses meshes whose largest
// remaining span (recon_span_bytes) reaches 4 GiB.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, uint64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0,
                                             int(bytes < 0xffffffffull ? uint32_t(bytes) : 0xffffffffu), 0x00020000);
}
// Descriptor of `rows` rows of n_cell entries starting at row `row` of a
// cell-fastest array (64-bit base arithmetic in scalar registers).
template <class E>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const E* base, int64_t row, int64_t nc, int rows = 1) {
    return rsrc(base + row * nc, uint64_t(rows) * uint64_t(nc) * sizeof(E));
}
template <class T>
__device__ __forceinline__ T bld(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, int(voff), int(soff), 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, int(voff), int(soff), 0));
}
// f(integral_constant<int, I>) for I = 0 .. N-1, unrolled at compile time
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <class T>
__device__ __forceinline__ void bst(T val, __amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, val), rs, int(voff), int(soff), 0);
    else
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, val), rs, int(voff), int(soff), 0);
}

// a = B_c b over the central stencil.  With FEAT, js[] also receives the max
// and the sum of |b| for rho (js[0], js[1]) and rho E (js[2], js[3]), which
// the gate features use (padding members contribute zero jumps).
//
// MCw (wave-uniform, at most MC) bounds the member loop: the largest central
// stencil among the wave's cells (slots past a cell's own stencil hold zero
// operator rows and the cell itself, so they add nothing).
template <class T, int K, bool FEAT = false>
__device__ __forceinline__ void central_coeffs(const ReconArgs<T>& A, int64_t c, const double* ui, T a[K][5],
                                               T* js = nullptr, int MCw = 0) {
    const int64_t nc = A.nc;
    const int MC = MCw > 0 && MCw < A.MC ? MCw : A.MC;
    // member m's id at sten_c[m][c]; its K operator rows at Bc[m][k][c]; U[v][j]
    const uint32_t rowT = uint32_t(nc) * uint32_t(sizeof(T)), rowU = uint32_t(nc) * 8u;
    const uint32_t c4 = uint32_t(c) * 4u, cT = uint32_t(c) * uint32_t(sizeof(T));
    const auto rU = rsrc(A.U, uint64_t(5) * rowU);
    auto member_id = [&](int m) { return bld<int32_t>(row_rsrc(A.sten_c, m, nc), c4, 0u); };
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int v = 0; v < 5; ++v) a[k][v] = T(0);
    if constexpr (FEAT) js[0] = js[1] = js[2] = js[3] = T(0);
    if constexpr (K <= 9) {
        // Loads run DEPTH members ahead of the arithmetic (three in FP32, two in
        // FP64: the kernels' register peak is in the directional phase, so this
        // costs no occupancy) and member ids R = DEPTH + 1 members further still,
        // so a state load finds its id loaded a whole trip earlier.  Member m
        // sits in slot m % R; the loop advances R members per trip with
        // compile-time slots (no register is copied while its load is in flight)
        // and a scheduling barrier after each member (the scheduler would
        // otherwise gather the trip's arithmetic at its top and wait there for
        // every load in flight).
        constexpr int DEPTH = sizeof(T) == 4 ? 3 : 2;
        constexpr int R = DEPTH + 1;
        auto last = [&](int m) { return m < MC ? m : MC - 1; };
        double u[R][5];
        T b[R][K];
        int32_t jr[R];  // id slot s: member m + DEPTH with (m + DEPTH) % R == s
        auto load_member = [&](int m, int32_t j, double* uu, T* bb) {
#pragma unroll
            for (int v = 0; v < 5; ++v) uu[v] = bld<double>(rU, uint32_t(j) * 8u, uint32_t(v) * rowU);
            const auto rB = row_rsrc(A.Bc, int64_t(last(m)) * K, nc, K);
#pragma unroll
            for (int k = 0; k < K; ++k) bb[k] = bld<T>(rB, cT, uint32_t(k) * rowT);
        };
#pragma unroll
        for (int d = 0; d < DEPTH + R; ++d) {
            const int32_t j = member_id(last(d));
            if (d < DEPTH)
                load_member(d, j, u[d], b[d]);
            else
                jr[d % R] = j;
        }
#pragma unroll 1
        for (int m0 = 0; m0 < MC; m0 += R) {
            static_for<0, R>([&](auto S) {
                constexpr int SL = decltype(S)::value, SD = (SL + DEPTH) % R;
                const int m = m0 + SL;
                // issue member m+DEPTH (operands) and the id of member m+DEPTH+R
                const int32_t j = jr[SD];
                jr[SD] = member_id(last(m + DEPTH + R));
                load_member(m + DEPTH, j, u[SD], b[SD]);
                if (m < MC) {  // uniform
                    T bv[5];
#pragma unroll
                    for (int v = 0; v < 5; ++v) bv[v] = T(u[SL][v] - ui[v]);
                    if constexpr (FEAT) {
                        js[0] = fmax(js[0], fabs(bv[0]));
                        js[1] += fabs(bv[0]);
                        js[2] = fmax(js[2], fabs(bv[4]));
                        js[3] += fabs(bv[4]);
                    }
#pragma unroll
                    for (int k = 0; k < K; ++k)
#pragma unroll
                        for (int v = 0; v < 5; ++v) a[k][v] += b[SL][k] * bv[v];
                }
                __builtin_amdgcn_sched_barrier(0);
            });
        }
    } else {
        // P3 (19 terms, one wave per SIMD in FP64): the loop unrolled by the
        // compiler with the register ring shifted each member measured faster
        // than fixed slots with a barrier per member.
        // Loads run DEPTH members ahead of the arithmetic (member ids one further):
        // three in FP32, two in FP64 (the kernels' register peak is in the
        // directional phase, so this costs no occupancy).
        constexpr int DEPTH = sizeof(T) == 4 ? 3 : 2;
        auto last = [&](int m) { return m < MC ? m : MC - 1; };
        double u[DEPTH + 1][5];
        T b[DEPTH + 1][K];
        int32_t jn[DEPTH + 1];  // ids of members m+1 .. m+DEPTH+1 (jn[0] unused after the prologue)
#pragma unroll
        for (int d = 0; d <= DEPTH; ++d) jn[d] = member_id(last(d));
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) {
#pragma unroll
            for (int v = 0; v < 5; ++v) u[d][v] = bld<double>(rU, uint32_t(jn[d]) * 8u, uint32_t(v) * rowU);
            const auto rB = row_rsrc(A.Bc, int64_t(last(d)) * K, nc, K);
#pragma unroll
            for (int k = 0; k < K; ++k) b[d][k] = bld<T>(rB, cT, uint32_t(k) * rowT);
        }
        int32_t jnext = jn[DEPTH];  // id of member DEPTH
#pragma unroll DEPTH + 1
        for (int m = 0; m < MC; ++m) {
            // issue member m+DEPTH (operands) and the id of member m+DEPTH+1
            const int mf = last(m + DEPTH);
            const int32_t jf = member_id(last(m + DEPTH + 1));
#pragma unroll
            for (int v = 0; v < 5; ++v) u[DEPTH][v] = bld<double>(rU, uint32_t(jnext) * 8u, uint32_t(v) * rowU);
            {
                const auto rB = row_rsrc(A.Bc, int64_t(mf) * K, nc, K);
#pragma unroll
                for (int k = 0; k < K; ++k) b[DEPTH][k] = bld<T>(rB, cT, uint32_t(k) * rowT);
            }
            // member m
            T bv[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) bv[v] = T(u[0][v] - ui[v]);
            if constexpr (FEAT) {
                js[0] = fmax(js[0], fabs(bv[0]));
                js[1] += fabs(bv[0]);
                js[2] = fmax(js[2], fabs(bv[4]));
                js[3] += fabs(bv[4]);
            }
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int v = 0; v < 5; ++v) a[k][v] += b[0][k] * bv[v];
#pragma unroll
            for (int d = 0; d < DEPTH; ++d) {
#pragma unroll
                for (int v = 0; v < 5; ++v) u[d][v] = u[d + 1][v];
#pragma unroll
                for (int k = 0; k < K; ++k) b[d][k] = b[d + 1][k];
            }
            jnext = jf;
        }
    }
}

// Largest central stencil among the wave's cells (every lane of the wave
// calls this; lanes past the mesh count zero).
template <class T>
__device__ __forceinline__ int wave_max_ncen(const ReconArgs<T>& A, int64_t c, bool valid) {
    int v = int(A.ncen[valid ? c : 0]);  // unconditional load (a lane condition would make it wait)
    v = valid ? v : 0;
    const int lane = int(threadIdx.x & 63u);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) v = max(v, __builtin_amdgcn_ds_bpermute((lane ^ d) << 2, v));
    return __builtin_amdgcn_readfirstlane(v);
}

// Twelve gate features of a cell, for v in (rho, rho E): log(1e-12 + x) of
//  (1) max and (2) mean of |v_m - v_i| / |v_i| over the central stencil,
//  (3) h |grad p_opt| / |v_i| (the central polynomial's gradient at the
//      centroid is a_lin / h),
//  (4-6) max, mean and min over the face neighbours j of
//      |v_j - v_i - grad p_opt . (c_j - c_i)| / (|v_j - v_i| + h |grad p_opt| + 1e-12 |v_i|).
template <class T>
__device__ __forceinline__ T feat_log(T x) {
    // the features feed a BF16 network: FP32 takes the hardware logarithm
    if constexpr (sizeof(T) == 4)
        return __logf(x);
    else
        return log(x);
}

template <class T, int K>
__device__ __forceinline__ void gate_features(const ReconArgs<T>& A, int64_t c, const double* ui, const T a[K][5],
                                              const T* js, float* f) {
    const int64_t nc = A.nc;
    const T h = A.hb[c], ninv = T(1) / T(A.ncen[c]);
    T au[2], g[2][3], gn[2], dmax[2], dsum[2], dmin[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int v = t ? 4 : 0;
        au[t] = fabs(T(ui[v]));
#pragma unroll
        for (int d = 0; d < 3; ++d) g[t][d] = a[d][v];
        gn[t] = sqrt(g[t][0] * g[t][0] + g[t][1] * g[t][1] + g[t][2] * g[t][2]);
        dmax[t] = dsum[t] = T(0);
        dmin[t] = T(INFINITY);
    }
    // one pass over the face neighbours for both variables; all their ids,
    // offsets and states are loaded up front (two memory round trips in all)
    const int NF = A.NF;
    const uint32_t rowI = uint32_t(nc) * 4u, rowT = uint32_t(nc) * uint32_t(sizeof(T)), rowU = uint32_t(nc) * 8u;
    const uint32_t c4 = uint32_t(c) * 4u, cT = uint32_t(c) * uint32_t(sizeof(T));
    const auto rN = rsrc(A.nbr, uint64_t(NF) * rowI);
    const auto rU = rsrc(A.U, uint64_t(5) * rowU);
    int32_t jn[kMaxFaces];
    T dn[kMaxFaces][3];
    double un[kMaxFaces][2];
#pragma unroll
    for (int lf = 0; lf < kMaxFaces; ++lf) {
        jn[lf] = lf < NF ? bld<int32_t>(rN, c4, uint32_t(lf) * rowI) : -1;
#pragma unroll
        for (int d = 0; d < 3; ++d)
            dn[lf][d] = lf < NF ? bld<T>(row_rsrc(A.ndc, int64_t(lf) * 3, nc, 3), cT, uint32_t(d) * rowT) : T(0);
    }
#pragma unroll
    for (int lf = 0; lf < kMaxFaces; ++lf)
#pragma unroll
        for (int t = 0; t < 2; ++t)
            un[lf][t] = bld<double>(rU, uint32_t(jn[lf] >= 0 ? jn[lf] : 0) * 8u, uint32_t(t ? 4 : 0) * rowU);
    int cnt = 0;
#pragma unroll
    for (int lf = 0; lf < kMaxFaces; ++lf) {
        if (jn[lf] < 0) continue;
        const T dx = dn[lf][0], dy = dn[lf][1], dz = dn[lf][2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int v = t ? 4 : 0;
            const T du = T(un[lf][t] - ui[v]);
            const T rr = fabs(du - (g[t][0] * dx + g[t][1] * dy + g[t][2] * dz) / h) /
                         (fabs(du) + gn[t] + T(1e-12) * au[t]);
            dmax[t] = fmax(dmax[t], rr);
            dmin[t] = fmin(dmin[t], rr);
            dsum[t] += rr;
        }
        ++cnt;
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        float* o = f + 6 * t;
        o[0] = float(feat_log(T(1e-12) + js[2 * t] / au[t]));
        o[1] = float(feat_log(T(1e-12) + js[2 * t + 1] * ninv / au[t]));
        o[2] = float(feat_log(T(1e-12) + gn[t] / au[t]));
        o[3] = float(feat_log(T(1e-12) + dmax[t]));
        o[4] = float(feat_log(T(1e-12) + dsum[t] / T(cnt > 0 ? cnt : 1)));
        o[5] = float(feat_log(T(1e-12) + (cnt > 0 ? dmin[t] : T(0))));
    }
}

// Steps per cell:
//  (i)   stencil jumps b_m = U_m - U_i in FP64, rounded to T
//  (ii)  a_opt = B_c b
//  (iii) a_s = B_s b_s per directional (linear) stencil
//  (iv)  SI_1 = a_opt^T O a_opt, SI_s = a_s^T O_lin a_s
//  (v)   tau = mean |SI_1 - SI_s|, w~ = lambda (1 + tau/(eps + SI))
//  (vi)  Levy-Puppo-Russo blend accumulated in one pass over the stencils:
//        abar = s1 a_opt + (tau/W) G on the linear modes, with
//        s1 = (1 + tau/(eps+SI_1))/W, W = 1 + tau sum_s lambda_s/(eps+SI_s),
//        G = sum_{s>=2} lambda_s (1/(eps+SI_s) - 1/(eps+SI_1)) a_s
//  (vii) point values U_i + Phi_q . abar at the cell's face points, with the
//        positivity fallback linear -> CWENOZ -> first order.

// SI_1 = a^T O a with O stored as its upper triangle; a sum of squares, so a
// rounded value below zero is rounding only and is clamped.
template <class T, int K>
__device__ __forceinline__ void si_opt(const ReconArgs<T>& A, int64_t c, const T a[K][5], T SI1[5]) {
    const int64_t nc = A.nc;
#pragma unroll
    for (int v = 0; v < 5; ++v) SI1[v] = T(0);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const T okk = A.O[int64_t(tri_index(K, k, k)) * nc + c];
        T t[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) t[v] = okk * a[k][v];
#pragma unroll
        for (int l = k + 1; l < K; ++l) {
            const T o2 = T(2) * A.O[int64_t(tri_index(K, k, l)) * nc + c];
#pragma unroll
            for (int v = 0; v < 5; ++v) t[v] += o2 * a[l][v];
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) SI1[v] += a[k][v] * t[v];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) SI1[v] = fmax(SI1[v], T(0));
}

// Basis functions at a face point from its offset (x, y, z) in the cell's
// scaled frame: the monomials of degree 1..r in graded-lex order (x exponent
// descending, then y) minus their cell means pm.  Recomputing them costs a
// few multiplies and reads 3 values per point instead of K.
template <class T, int K>
__device__ __forceinline__ void basis_at(T x, T y, T z, const T* pm, T* ph) {
    ph[0] = x - pm[0];
    ph[1] = y - pm[1];
    ph[2] = z - pm[2];
    if constexpr (K >= 9) {
        ph[3] = x * x - pm[3];
        ph[4] = x * y - pm[4];
        ph[5] = x * z - pm[5];
        ph[6] = y * y - pm[6];
        ph[7] = y * z - pm[7];
        ph[8] = z * z - pm[8];
    }
    if constexpr (K >= 19) {
        const T xx = x * x, yy = y * y, zz = z * z;
        ph[9] = xx * x - pm[9];
        ph[10] = xx * y - pm[10];
        ph[11] = xx * z - pm[11];
        ph[12] = x * yy - pm[12];
        ph[13] = x * y * z - pm[13];
        ph[14] = x * zz - pm[14];
        ph[15] = yy * y - pm[15];
        ph[16] = yy * z - pm[16];
        ph[17] = y * zz - pm[17];
        ph[18] = zz * z - pm[18];
    }
}

// Most Gauss points on one face for a basis of K terms (order p: p*p on a
// quadrilateral, 3 on a triangle); the launcher rejects meshes beyond it.
template <int K>
constexpr int face_qmax() { return K <= 9 ? 4 : 9; }
// Points of one face staged together in LDS before their stores (P2: a whole
// face, so one LDS round trip per face; P3: three at a time, a whole
// triangle).
template <int K>
constexpr int stage_points() { return face_qmax<K>() <= 4 ? face_qmax<K>() : 3; }

// Point values U_i + Phi(x_q) . a at the cell's face points (step vii) from
// the coefficients a (first order when mode == 2); returns whether density and
// pressure are positive at all of them.  Point states are stored per point
// slot (lf, q) as rows of [cell][5] (cells padded to whole 64-cell tiles), so
// that the flux kernel reads a cell's five values from one run.
// STAGE, in a wave whose 64 cells all exist (all its lanes here): each
// point's 64 x 5 values pass through the wave's LDS (320 values per point,
// stage_points<K>() points at a time) and leave as five contiguous 64-value
// stores; a lane without the point stores a value into its unused slot.
// Otherwise (the positivity fallback, the mesh's last, partial wave) each
// lane stores its own points' five values.
template <class T, int K, bool STAGE>
__device__ __forceinline__ bool face_values(const ReconArgs<T>& A, int64_t c, const double* ui, int mode,
                                            const T a[K][5], T* stage = nullptr) {
    const int64_t nc = A.nc;
    const int NF = A.NF, Q = A.Q;
    const uint32_t rowT = uint32_t(nc) * uint32_t(sizeof(T));
    const uint32_t cT = uint32_t(c) * uint32_t(sizeof(T));
    const int64_t ncp = fs_cells_padded(nc);
    const int lane = int(threadIdx.x & 63u);
    // element offsets (bytes) in a slot row: this lane's own cell, and this
    // lane's share of its wave's staged run
    const uint32_t cF = 5u * cT;
    const uint32_t wF = (uint32_t(c - lane) * 5u + uint32_t(lane)) * uint32_t(sizeof(T));
    const bool staged = STAGE && c - lane + 64 <= nc;  // wave-uniform
    T pm[K];
    {
        const auto rM = row_rsrc(A.pmean, 0, nc, K);
#pragma unroll
        for (int k = 0; k < K; ++k) pm[k] = bld<T>(rM, cT, uint32_t(k) * rowT);
    }
    bool ok = true;
    // The loops are wave-uniform (every lane walks all NF x Q slots); a lane
    // without the point (nq of the slot) skips it, or, staged, forms a value
    // that lands in its unused slot.  The offset of point (lf, q) in rows
    // ((lf Q + q) 3 + d).  The next face's offsets and point count load while
    // this face's points are formed, so only the first face waits on memory.
    constexpr int QM = face_qmax<K>();
    auto load_face = [&](int lf, T (&x)[QM][3]) {
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const auto rX = row_rsrc(A.xi, (int64_t(lf) * Q + q) * 3, nc, 3);
#pragma unroll
            for (int d = 0; d < 3; ++d) x[q][d] = q < Q ? bld<T>(rX, cT, uint32_t(d) * rowT) : T(0);
        }
        return int(__builtin_amdgcn_raw_buffer_load_b8(row_rsrc(A.cnq, lf, nc), int(uint32_t(c)), 0, 0));
    };
    T x[QM][3], xn[QM][3];
    int nq = load_face(0, x);
#pragma unroll 1
    for (int lf = 0; lf < NF; ++lf) {
        const int nqn = lf + 1 < NF ? load_face(lf + 1, xn) : 0;
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            if (q >= Q) continue;  // wave-uniform
            if (!staged && q >= nq) continue;
            T d[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) d[v] = T(0);
            if (mode != 2) {
                T ph[K];
                basis_at<T, K>(x[q][0], x[q][1], x[q][2], pm, ph);
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int v = 0; v < 5; ++v) d[v] += ph[k] * a[k][v];
            }
            T val[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) val[v] = T(ui[v] + double(d[v]));
            const T p = A.gm1 * (val[4] - T(0.5) * (val[1] * val[1] + val[2] * val[2] + val[3] * val[3]) / val[0]);
            if (q < nq) ok = ok && (val[0] > T(1e-10)) && (p > T(1e-10));
            if (staged) {
                constexpr int QB = stage_points<K>();
                const int sq = q % QB;  // a constant once the point loop is unrolled
#pragma unroll
                for (int v = 0; v < 5; ++v) stage[sq * 320 + lane * 5 + v] = val[v];
                if (sq == QB - 1 || q == Q - 1) {  // wave-uniform: flush the batch
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int b = 0; b <= sq; ++b) {
                        const auto rF = row_rsrc(A.fs, (int64_t(lf) * Q + q - sq + b) * 5, ncp, 5);
#pragma unroll
                        for (int k = 0; k < 5; ++k)
                            bst<T>(stage[b * 320 + k * 64 + lane], rF, wF, uint32_t(k) * 64u * uint32_t(sizeof(T)));
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            } else {
                const auto rF = row_rsrc(A.fs, (int64_t(lf) * Q + q) * 5, ncp, 5);
#pragma unroll
                for (int v = 0; v < 5; ++v) bst<T>(val[v], rF, cF, uint32_t(v) * uint32_t(sizeof(T)));
            }
        }
#pragma unroll
        for (int q = 0; q < QM; ++q)
#pragma unroll
            for (int d = 0; d < 3; ++d) x[q][d] = xn[q][d];
        nq = nqn;
    }
    return ok;
}

// Running state of the blend (steps iv-vi) of one cell: the central
// indicator, the sums over its directional stencils and the linear-mode
// correction G, so that stencils can be added one at a time.
template <class T>
struct Blend {
    T lam_s, lam_1;
    T SI1[5], inv1[5], tsum[5], Lam[5], rmin[5], rmax[5], g[3][5];
    T o00, o01, o02, o11, o12, o22;  // the linear block of O
};

template <class T, int K>
__device__ __forceinline__ void blend_init(const ReconArgs<T>& A, int64_t c, int nd, const T a[K][5], Blend<T>& B) {
    const int64_t nc = A.nc;
    B.lam_s = T(1) / (A.lam_c + T(nd));
    B.lam_1 = A.lam_c * B.lam_s;
    si_opt<T, K>(A, c, a, B.SI1);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        B.tsum[v] = T(0);
        B.inv1[v] = T(1) / (A.eps + B.SI1[v]);
        B.Lam[v] = B.lam_1 * B.inv1[v];
        B.rmin[v] = B.inv1[v];
        B.rmax[v] = B.inv1[v];
#pragma unroll
        for (int k = 0; k < 3; ++k) B.g[k][v] = T(0);
    }
    B.o00 = A.O[0 * nc + c];
    B.o01 = A.O[1 * nc + c];
    B.o02 = A.O[2 * nc + c];
    B.o11 = A.O[int64_t(K) * nc + c];
    B.o12 = A.O[int64_t(K + 1) * nc + c];
    B.o22 = A.O[int64_t(2 * K - 1) * nc + c];
}

// One directional stencil with linear coefficients as: its indicator and its
// share of the blend.
template <class T>
__device__ __forceinline__ void blend_add(const ReconArgs<T>& A, Blend<T>& B, const T as[3][5]) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        const T x = as[0][v], y = as[1][v], z = as[2][v];
        const T SIs = fmax(x * (B.o00 * x + T(2) * (B.o01 * y + B.o02 * z)) + y * (B.o11 * y + T(2) * B.o12 * z) +
                               z * B.o22 * z,
                           T(0));
        B.tsum[v] += fabs(B.SI1[v] - SIs);
        const T r = T(1) / (A.eps + SIs);
        B.Lam[v] += B.lam_s * r;
        B.rmin[v] = fmin(B.rmin[v], r);
        B.rmax[v] = fmax(B.rmax[v], r);
        const T coef = B.lam_s * (r - B.inv1[v]);
#pragma unroll
        for (int k = 0; k < 3; ++k) B.g[k][v] += coef * as[k][v];
    }
}

// The blended coefficients (overwriting the central ones in a) and, with
// LABEL, max |omega - lambda| over variables and stencils.
template <class T, int K, bool LABEL>
__device__ __forceinline__ void blend_finish(Blend<T>& B, int nd, float& lab, T a[K][5]) {
    T s1[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        const T tau = B.tsum[v] / T(nd);
        const T W = T(1) + tau * B.Lam[v];
        s1[v] = (T(1) + tau * B.inv1[v]) / W;
        const T tw = tau / W;
#pragma unroll
        for (int k = 0; k < 3; ++k) B.g[k][v] *= tw;
        if constexpr (LABEL) {
            // |omega_s - lambda_s| = lambda_s |(1 + tau r_s)/W - 1|: extreme at rmin or rmax
            const float d1 = float(fabs(B.lam_1 * (s1[v] - T(1))));
            const float d2 = float(fabs(B.lam_s * ((T(1) + tau * B.rmin[v]) / W - T(1))));
            const float d3 = float(fabs(B.lam_s * ((T(1) + tau * B.rmax[v]) / W - T(1))));
            lab = fmaxf(lab, fmaxf(d1, fmaxf(d2, d3)));
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int v = 0; v < 5; ++v) a[k][v] = s1[v] * a[k][v] + (k < 3 ? B.g[k < 3 ? k : 0][v] : T(0));
}

// One lane per cell: steps (iii)-(vi) for a cell with nd > 0 directional
// stencils.  a holds the central coefficients on entry; it is overwritten by
// the blend.
template <class T, int K, bool LABEL>
__device__ __forceinline__ void dir_blend_lane(const ReconArgs<T>& A, int64_t c, const double* ui, int nd, float& lab,
                                               T a[K][5]) {
    const int64_t nc = A.nc;
    Blend<T> B;
    blend_init<T, K>(A, c, nd, a, B);
    // all directional members as one pipelined stream t = s * MD + m over
    // every stencil slot (a wave-uniform count; the slots past the cell's
    // nd hold zero operators and are not counted); the id of member t at
    // sten_d[t][c], its 3 operator rows at Bd[t][k][c]
    const int MD = A.MD, total = A.ND * MD;
    const uint32_t rowT = uint32_t(nc) * uint32_t(sizeof(T));
    const uint32_t rowU = uint32_t(nc) * 8u;
    const uint32_t c4 = uint32_t(c) * 4u, cT = uint32_t(c) * uint32_t(sizeof(T));
    const auto rU = rsrc(A.U, uint64_t(5) * rowU);
    auto member_id = [&](int t) { return bld<int32_t>(row_rsrc(A.sten_d, t, nc), c4, 0u); };
    if constexpr (K <= 9) {
        // loads DEPTH members ahead and ids R = DEPTH + 1 further, in trips of R
        // members with compile-time slots, as in central_coeffs
        constexpr int DEPTH = sizeof(T) == 4 ? 2 : 1;
        constexpr int R = DEPTH + 1;
        auto last = [&](int t) { return t < total ? t : total - 1; };
        double u[R][5];
        T b[R][3];
        int32_t jr[R];
        auto load_member = [&](int t, int32_t j, double* uu, T* bb) {
#pragma unroll
            for (int v = 0; v < 5; ++v) uu[v] = bld<double>(rU, uint32_t(j) * 8u, uint32_t(v) * rowU);
            const auto rB = row_rsrc(A.Bd, int64_t(last(t)) * 3, nc, 3);
#pragma unroll
            for (int k = 0; k < 3; ++k) bb[k] = bld<T>(rB, cT, uint32_t(k) * rowT);
        };
#pragma unroll
        for (int d = 0; d < DEPTH + R; ++d) {
            const int32_t j = member_id(last(d));
            if (d < DEPTH)
                load_member(d, j, u[d], b[d]);
            else
                jr[d % R] = j;
        }
        T as[3][5];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int v = 0; v < 5; ++v) as[k][v] = T(0);
        int m = 0, s = 0;
#pragma unroll 1
        for (int t0 = 0; t0 < total; t0 += R) {
            static_for<0, R>([&](auto S) {
                constexpr int SL = decltype(S)::value, SD = (SL + DEPTH) % R;
                const int t = t0 + SL;
                const int32_t j = jr[SD];
                jr[SD] = member_id(last(t + DEPTH + R));
                load_member(t + DEPTH, j, u[SD], b[SD]);
                if (t < total) {  // uniform
                    T bv[5];
#pragma unroll
                    for (int v = 0; v < 5; ++v) bv[v] = T(u[SL][v] - ui[v]);
#pragma unroll
                    for (int k = 0; k < 3; ++k)
#pragma unroll
                        for (int v = 0; v < 5; ++v) as[k][v] += b[SL][k] * bv[v];
                    if (m + 1 == MD) {
                        // stencil s complete
                        if (s < nd) blend_add<T>(A, B, as);
#pragma unroll
                        for (int k = 0; k < 3; ++k)
#pragma unroll
                            for (int v = 0; v < 5; ++v) as[k][v] = T(0);
                        m = 0;
                        ++s;
                    } else {
                        ++m;
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            });
        }
    } else {
        // P3: the compiler-unrolled ring, as in central_coeffs
        // loads DEPTH members ahead (ids one further), as in central_coeffs
        constexpr int DEPTH = sizeof(T) == 4 ? 2 : 1;
        auto last = [&](int t) { return t < total ? t : total - 1; };
        double u[DEPTH + 1][5];
        T b[DEPTH + 1][3];
        int32_t jn[DEPTH + 1];
#pragma unroll
        for (int d = 0; d <= DEPTH; ++d) jn[d] = member_id(last(d));
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) {
#pragma unroll
            for (int v = 0; v < 5; ++v) u[d][v] = bld<double>(rU, uint32_t(jn[d]) * 8u, uint32_t(v) * rowU);
            const auto rB = row_rsrc(A.Bd, int64_t(last(d)) * 3, nc, 3);
#pragma unroll
            for (int k = 0; k < 3; ++k) b[d][k] = bld<T>(rB, cT, uint32_t(k) * rowT);
        }
        int32_t jnext = jn[DEPTH];
        T as[3][5];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int v = 0; v < 5; ++v) as[k][v] = T(0);
        int m = 0, s = 0;
#pragma unroll 1
        for (int t = 0; t < total; ++t) {
            const int tf = last(t + DEPTH);
            const int32_t jf = member_id(last(t + DEPTH + 1));
#pragma unroll
            for (int v = 0; v < 5; ++v) u[DEPTH][v] = bld<double>(rU, uint32_t(jnext) * 8u, uint32_t(v) * rowU);
            {
                const auto rB = row_rsrc(A.Bd, int64_t(tf) * 3, nc, 3);
#pragma unroll
                for (int k = 0; k < 3; ++k) b[DEPTH][k] = bld<T>(rB, cT, uint32_t(k) * rowT);
            }
            T bv[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) bv[v] = T(u[0][v] - ui[v]);
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int v = 0; v < 5; ++v) as[k][v] += b[0][k] * bv[v];
            if (m + 1 == MD) {
                // stencil s complete
                if (s < nd) blend_add<T>(A, B, as);
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int v = 0; v < 5; ++v) as[k][v] = T(0);
                m = 0;
                ++s;
            } else {
                ++m;
            }
#pragma unroll
            for (int d = 0; d < DEPTH; ++d) {
#pragma unroll
                for (int v = 0; v < 5; ++v) u[d][v] = u[d + 1][v];
#pragma unroll
                for (int k = 0; k < 3; ++k) b[d][k] = b[d + 1][k];
            }
            jnext = jf;
        }
    }
    blend_finish<T, K, LABEL>(B, nd, lab, a);
}

// value of x in lane `lane` (wave-uniform index), read into every lane
template <class T>
__device__ __forceinline__ T lane_read(T x, int lane) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), lane));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, x);
        const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(u)), lane));
        const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(u >> 32)), lane));
        return __builtin_bit_cast(T, (uint64_t(hi) << 32) | lo);
    }
}

// value of lane (this lane + d), any lane of the wave (wraps past 63)
template <class T>
__device__ __forceinline__ T lane_down(T x, int lane, int d) {
    const int addr = ((lane + d) & 63) << 2;
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, x)));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, x);
        const uint32_t lo = uint32_t(__builtin_amdgcn_ds_bpermute(addr, int(uint32_t(u))));
        const uint32_t hi = uint32_t(__builtin_amdgcn_ds_bpermute(addr, int(uint32_t(u >> 32))));
        return __builtin_bit_cast(T, (uint64_t(hi) << 32) | lo);
    }
}

// Waves with at most this many troubled cells take them one at a time with
// the whole wave (dir_blend_wave); busier waves take dir_blend_stencils or
// one lane per cell.
constexpr int kWaveBlendMax = 2;

// Steps (iii)-(vi) for the troubled cells of a wave that has few of them
// (the lanes set in todo; every lane of the wave calls this).  One at a
// time, lane t loads directional slot t of the cell (stencil t / MD, member
// t % MD; ND * MD <= 64), the member products are summed per stencil across
// the lanes, and each stencil's coefficients are read by the cell's own lane,
// which forms the blend exactly as the one-lane path does.  A lone troubled
// cell thus waits for one round of loads instead of ND * MD of them.  Only
// the products' summation order differs from dir_blend_lane.
template <class T, int K>
__device__ __forceinline__ void dir_blend_wave(const ReconArgs<T>& A, uint64_t todo, int64_t c, const double* ui,
                                               int nd, T a[K][5]) {
    const int64_t nc = A.nc;
    const int lane = int(threadIdx.x & 63u);
    const int MD = A.MD, total = A.ND * MD, m = lane % MD;
    const bool mine = (todo >> lane) & 1u;
    Blend<T> B;
    if (mine) blend_init<T, K>(A, c, nd, a, B);
    while (todo) {
        const int L = __builtin_ctzll(todo);
        todo &= todo - 1;
        const int64_t cL = __builtin_amdgcn_readlane(int(c), L);
        const int ndL = __builtin_amdgcn_readlane(nd, L);
        T x[3][5];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int v = 0; v < 5; ++v) x[k][v] = T(0);
        if (lane < total) {
            const int32_t j = A.sten_d[int64_t(lane) * nc + cL];
            T b[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) b[k] = A.Bd[(int64_t(lane) * 3 + k) * nc + cL];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const T bv = T(A.U[v * nc + j] - lane_read(ui[v], L));
#pragma unroll
                for (int k = 0; k < 3; ++k) x[k][v] = b[k] * bv;
            }
        }
        // sums over the members of each stencil: after the step with d,
        // lane s MD + m holds the sum over members m .. min(m + 2d, MD) - 1
        for (int d = 1; d < MD; d <<= 1) {
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    const T y = lane_down(x[k][v], lane, d);
                    if (m + d < MD) x[k][v] += y;
                }
        }
        for (int s = 0; s < ndL; ++s) {
            T as[3][5];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int v = 0; v < 5; ++v) as[k][v] = lane_read(x[k][v], s * MD);
            if (lane == L) blend_add<T>(A, B, as);
        }
    }
    float lab = 0.f;
    if (mine) blend_finish<T, K, false>(B, nd, lab, a);
}

// Busier waves (up to this many troubled cells) take their troubled cells
// with one lane per (cell, directional stencil); FP32 P2 only, where the
// central coefficients of a wave fit in its LDS.
constexpr int kStencilLanesMax = 30;

// value of x in lane src (any lane of the wave, per-lane index)
template <class T>
__device__ __forceinline__ T lane_from(T x, int src) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_ds_bpermute(src << 2, __builtin_bit_cast(int, x)));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, x);
        const uint32_t lo = uint32_t(__builtin_amdgcn_ds_bpermute(src << 2, int(uint32_t(u))));
        const uint32_t hi = uint32_t(__builtin_amdgcn_ds_bpermute(src << 2, int(uint32_t(u >> 32))));
        return __builtin_bit_cast(T, (uint64_t(hi) << 32) | lo);
    }
}

// Steps (iii)-(vi) for the troubled cells of a wave (the lanes set in todo;
// every lane of the wave calls this) with one lane per (cell, stencil): each
// pass gives the next 64 / ND troubled cells ND lanes each; lane s of a cell
// streams the MD members of the cell's stencil s and forms that stencil's
// indicator and blend terms, the terms are summed over the cell's lanes, and
// the cell's own lane adds them to its blend.  A troubled cell thus waits
// for MD member loads instead of ND * MD.  The lanes' central coefficients
// wait in LDS (stash, K * 5 * 64 floats) meanwhile, freeing their registers
// for the streams.  Only the summation order of the blend terms differs from
// dir_blend_lane.
template <int K, int SDEPTH = 2>
__device__ __forceinline__ void dir_blend_stencils(const ReconArgs<float>& A, uint64_t todo, int64_t c,
                                                   const double* ui, int nd, float a[K][5], float* stash) {
    using T = float;
    const int64_t nc = A.nc;
    const int lane = int(threadIdx.x & 63u);
    const int ND = A.ND, MD = A.MD, per = 64 / ND;
    const int p = lane / ND, s = lane - p * ND;  // this lane's cell (within the pass) and stencil
    const bool mine = (todo >> lane) & 1u;
    Blend<T> B;
    if (mine) blend_init<T, K>(A, c, nd, a, B);
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int v = 0; v < 5; ++v) stash[(k * 5 + v) * 64 + lane] = a[k][v];
    while (todo) {
        // the next `per` troubled cells, and this lane's cell among them
        uint64_t pass = 0, rest = todo;
        int src = -1;
        for (int k = 0; k < per && rest; ++k) {
            const int L = __builtin_ctzll(rest);
            pass |= 1ull << L;
            rest &= rest - 1;
            if (k == p) src = L;
        }
        todo = rest;
        const int sl = src >= 0 ? src : lane;
        const int cp = lane_from(int(c), sl);
        const int ndp = lane_from(nd, sl);
        const bool work = src >= 0 && s < ndp;
        double up[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) up[v] = lane_from(ui[v], sl);
        const int64_t cq = cp;
        T as[3][5];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int v = 0; v < 5; ++v) as[k][v] = T(0);
        if (work) {
            // members of stencil s, loads SDEPTH members ahead (ids one further)
            const int64_t r0 = int64_t(s) * MD;
            auto row = [&](int m) { return r0 + (m < MD ? m : MD - 1); };
            double u[SDEPTH + 1][5];
            T b[SDEPTH + 1][3];
            int32_t jn[SDEPTH + 1];
#pragma unroll
            for (int d = 0; d <= SDEPTH; ++d) jn[d] = A.sten_d[row(d) * nc + cq];
#pragma unroll
            for (int d = 0; d < SDEPTH; ++d) {
#pragma unroll
                for (int v = 0; v < 5; ++v) u[d][v] = A.U[v * nc + jn[d]];
#pragma unroll
                for (int k = 0; k < 3; ++k) b[d][k] = A.Bd[(row(d) * 3 + k) * nc + cq];
            }
            int32_t jnext = jn[SDEPTH];
#pragma unroll 1
            for (int m = 0; m < MD; ++m) {
                const int32_t jf = A.sten_d[row(m + SDEPTH + 1) * nc + cq];
#pragma unroll
                for (int v = 0; v < 5; ++v) u[SDEPTH][v] = A.U[v * nc + jnext];
#pragma unroll
                for (int k = 0; k < 3; ++k) b[SDEPTH][k] = A.Bd[(row(m + SDEPTH) * 3 + k) * nc + cq];
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    const T bv = T(u[0][v] - up[v]);
#pragma unroll
                    for (int k = 0; k < 3; ++k) as[k][v] += b[0][k] * bv;
                }
#pragma unroll
                for (int d = 0; d < SDEPTH; ++d) {
#pragma unroll
                    for (int v = 0; v < 5; ++v) u[d][v] = u[d + 1][v];
#pragma unroll
                    for (int k = 0; k < 3; ++k) b[d][k] = b[d + 1][k];
                }
                jnext = jf;
            }
        }
        // the stencil's indicator and blend terms (zero on idle lanes)
        T SI1p[5], inv1p[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            SI1p[v] = lane_from(B.SI1[v], sl);
            inv1p[v] = lane_from(B.inv1[v], sl);
        }
        T ts[5], lm[5], gg[3][5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            ts[v] = lm[v] = T(0);
#pragma unroll
            for (int k = 0; k < 3; ++k) gg[k][v] = T(0);
        }
        if (work) {
            const T o00 = A.O[0 * nc + cq], o01 = A.O[1 * nc + cq], o02 = A.O[2 * nc + cq];
            const T o11 = A.O[int64_t(K) * nc + cq], o12 = A.O[int64_t(K + 1) * nc + cq];
            const T o22 = A.O[int64_t(2 * K - 1) * nc + cq];
            const T lam_s = T(1) / (A.lam_c + T(ndp));
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const T x = as[0][v], y = as[1][v], z = as[2][v];
                const T SIs = fmax(x * (o00 * x + T(2) * (o01 * y + o02 * z)) + y * (o11 * y + T(2) * o12 * z) +
                                       z * o22 * z,
                                   T(0));
                ts[v] = fabs(SI1p[v] - SIs);
                const T r = T(1) / (A.eps + SIs);
                lm[v] = lam_s * r;
                const T coef = lam_s * (r - inv1p[v]);
#pragma unroll
                for (int k = 0; k < 3; ++k) gg[k][v] = coef * as[k][v];
            }
        }
        // sums over the ND lanes of each cell: after the step with d, lane
        // p ND + s holds the sum over stencils s .. min(s + 2d, ND) - 1
        for (int d = 1; d < ND; d <<= 1) {
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const T y0 = lane_down(ts[v], lane, d), y1 = lane_down(lm[v], lane, d);
                if (s + d < ND) {
                    ts[v] += y0;
                    lm[v] += y1;
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const T y = lane_down(gg[k][v], lane, d);
                    if (s + d < ND) gg[k][v] += y;
                }
            }
        }
        // each cell's lane takes its sums from lane rank * ND
        const bool inpass = (pass >> lane) & 1u;
        const int rank = int(__builtin_amdgcn_mbcnt_hi(uint32_t(pass >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(pass), 0u)));
        const int from = inpass ? rank * ND : lane;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const T x0 = lane_from(ts[v], from), x1 = lane_from(lm[v], from);
            if (inpass) {
                B.tsum[v] += x0;
                B.Lam[v] += x1;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const T x = lane_from(gg[k][v], from);
                if (inpass) B.g[k][v] += x;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int v = 0; v < 5; ++v) a[k][v] = stash[(k * 5 + v) * 64 + lane];
    float lab = 0.f;
    if (mine) blend_finish<T, K, false>(B, nd, lab, a);
}

// One lane per cell: steps (iii)-(vi) for mode 1, then (vii) for any mode
// (STAGE: the main pass; the positivity fallback runs on scattered cells and
// stores its own points).
template <class T, int K, bool LABEL, bool STAGE = false>
__device__ __forceinline__ bool recon_cell(const ReconArgs<T>& A, int64_t c, const double* ui, int mode, float& lab,
                                           T a[K][5], T* stage = nullptr) {
    if (mode == 1) {
        const int nd = A.ndir[c];
        if (nd > 0) dir_blend_lane<T, K, LABEL>(A, c, ui, nd, lab, a);
    }
    return face_values<T, K, STAGE>(A, c, ui, mode, a, stage);
}

// Main pass without a gate (full CWENOZ everywhere), or with a gate (a mask,
// or the troubled-cell network run inside this kernel).
//
// GATE: right after the central coefficients (which it needs anyway) each
// cell forms its features and the wave evaluates the network for its 64
// cells on the matrix cores, its weights read from the packed image (or it
// reads the mask).  Cells taken as smooth keep the linear central
// polynomial; the wave then finishes its troubled cells in this pass, by the
// whole wave one cell at a time (a few), one lane per (cell, stencil) (up to
// kStencilLanesMax, FP32 P2), or one lane per cell.  (Moving the troubled
// cells to a separate pass, a wave or a quad of lanes per cell, was measured
// slower: an isolated troubled cell then reads a cache line per operator
// value, while here its central and face data stream with its neighbours'.)
// The FP32 P2 variant is held to 3 waves per SIMD, which its LDS already
// imposes.
//
// A cell whose point states violate positivity is marked with bit 7 of its
// flag for the fallback pass.  GRAD (1 Green-Gauss, 2 least squares): the
// cell then forms its gradient of W as well (the positivity fallback changes
// point states only, never the cell averages the gradient is taken from).
template <class T, int K, bool LABEL, bool GATE, int GRAD = 0>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(
    K == 9 && (sizeof(T) == 4 ? GATE : !GATE && !LABEL) ? (sizeof(T) == 4 ? 3 : 2) : 1)))
void reconstruct_kernel(ReconArgs<T> A) {
    const int64_t c = xcd_block() * blockDim.x + threadIdx.x;
    const bool valid = c < A.nc;
    // the wave's largest central stencil (all lanes, before any divergence;
    // skipped when every cell has MC members)
    const int MCw = A.MCmin < A.MC ? wave_max_ncen(A, c, valid) : A.MC;
    double ui[5];
    T a[K][5];
    if constexpr (GATE) {
        int mode = 0;
        // per wave: the network's scratch, then (FP32 P2) the stash of
        // dir_blend_stencils
        constexpr int kStash = sizeof(T) == 4 && K == 9 ? K * 5 * 64 * 4 : 0;
        constexpr int kStage = stage_points<K>() * 320 * int(sizeof(T));  // then the point-state staging
        constexpr int kWaveLds0 = sizeof(MlpWaveLds) > kStash ? int(sizeof(MlpWaveLds)) : kStash;
        constexpr int kWaveLds = kWaveLds0 > kStage ? kWaveLds0 : kStage;
        __shared__ __attribute__((aligned(16))) unsigned char lds[kBlock / 64][kWaveLds];
        unsigned char* wl = lds[threadIdx.x >> 6];
        if (A.mlp) {
            const float* fv = reinterpret_cast<const float*>(A.mlp + mlpimg::kF);
            float f[12];
            if (valid) {
#pragma unroll
                for (int v = 0; v < 5; ++v) ui[v] = A.U[v * A.nc + c];
                T js[4];
                central_coeffs<T, K, true>(A, c, ui, a, js, MCw);
                gate_features<T, K>(A, c, ui, a, js, f);
            } else {
#pragma unroll
                for (int k = 0; k < 12; ++k) f[k] = fv[mlpimg::kMu + k];
            }
            const float z = mlp_wave_forward_packed(A.mlp, *reinterpret_cast<MlpWaveLds*>(wl), f);  // all lanes
            mode = 1.f / (1.f + __expf(-z)) < fv[mlpimg::kTheta] ? 0 : 1;
        } else if (valid) {
#pragma unroll
            for (int v = 0; v < 5; ++v) ui[v] = A.U[v * A.nc + c];
            central_coeffs<T, K>(A, c, ui, a, nullptr, MCw);
            mode = A.gate[c] ? 0 : 1;
        }
        // troubled cells: the whole wave per cell when the wave has few, one
        // lane per (cell, stencil) when it has more, else one lane per cell
        const int nd = valid && mode == 1 ? int(A.ndir[c]) : 0;
        const uint64_t todo = __builtin_amdgcn_ballot_w64(nd > 0);
        const int nt = __builtin_popcountll(todo);
        bool done = todo == 0;
        if (!done && nt <= kWaveBlendMax && A.ND * A.MD <= 64) {
            dir_blend_wave<T, K>(A, todo, c, ui, nd, a);
            done = true;
        }
        if constexpr (kStash > 0) {
            if (!done && nt <= kStencilLanesMax) {
                dir_blend_stencils<K>(A, todo, c, ui, nd, a, reinterpret_cast<float*>(wl));
                done = true;
            }
        }
        if (!done && nd > 0) {
            float lab = 0.f;
            dir_blend_lane<T, K, false>(A, c, ui, nd, lab, a);
        }
        if (!valid) return;
        if (A.mask_out) A.mask_out[c] = mode == 0 ? 1 : 0;
        // the network's LDS row is free again: it stages the point states
        const bool ok = face_values<T, K, true>(A, c, ui, 0, a, reinterpret_cast<T*>(wl));
        A.flags[c] = uint8_t((mode == 0 ? 1 : 0) | (ok ? 0 : 0x80));
        if constexpr (GRAD != 0) cell_gradient<T, GRAD == 2>(A, c, ui);
    } else {
        __shared__ T stage[kBlock / 64][stage_points<K>() * 320];
        if (!valid) return;
#pragma unroll
        for (int v = 0; v < 5; ++v) ui[v] = A.U[v * A.nc + c];
        central_coeffs<T, K>(A, c, ui, a, nullptr, MCw);
        float lab = 0.f;
        const bool ok = recon_cell<T, K, LABEL, true>(A, c, ui, 1, lab, a, stage[threadIdx.x >> 6]);
        A.flags[c] = uint8_t(ok ? 0 : 0x80);
        if constexpr (LABEL) A.label[c] = lab;
        if constexpr (GRAD != 0) cell_gradient<T, GRAD == 2>(A, c, ui);
    }
}

// Gate features only ([n_cell][12] float), from the central coefficients.
template <class T, int K>
__global__ __launch_bounds__(kBlock) void gate_features_kernel(ReconArgs<T> A, float* out) {
    const int64_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= A.nc) return;
    double ui[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) ui[v] = A.U[v * A.nc + c];
    T a[K][5], js[4];
    central_coeffs<T, K, true>(A, c, ui, a, js);
    float f[12];
    gate_features<T, K>(A, c, ui, a, js, f);
#pragma unroll
    for (int k = 0; k < 12; ++k) out[c * 12 + k] = f[k];
}

// Fallback pass over the marked cells: gated-linear -> full CWENOZ -> first
// order, rewriting the cell's point states (bit1 / bit2 record the steps).
template <class T, int K>
__global__ __launch_bounds__(kBlock) void reconstruct_fallback_kernel(ReconArgs<T> A) {
    const int64_t c = xcd_block() * blockDim.x + threadIdx.x;
    if (c >= A.nc) return;
    uint8_t fl = A.flags[c];
    if (!(fl & 0x80)) return;
    double ui[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) ui[v] = A.U[v * A.nc + c];
    int mode = (fl & 1) ? 0 : 1;
    fl &= 0x7f;
    float lab = 0.f;
    while (true) {
        fl |= mode == 0 ? 2 : 4;
        ++mode;
        T a[K][5];
        central_coeffs<T, K>(A, c, ui, a);
        if (recon_cell<T, K, false>(A, c, ui, mode, lab, a) || mode == 2) break;
    }
    A.flags[c] = fl;
}
