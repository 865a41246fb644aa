// P4 (CWENOZ5) reconstruction kernel (included by ucns_kernels.hip).
//
// Sec. 2.2 of the UCNS3D v4 paper at fifth order: a central polynomial of
// degree 4 (34 zero-mean basis terms) on the central stencil, one quadratic
// directional polynomial (9 terms) per face on a sectorial stencil, their
// smoothness indicators and WENO-Z weights (eq. cwenoz_weights), the CWENOZ
// blend (eq. cwenoz_poly, Levy-Puppo-Russo form) and the point values at the
// cell's 6 x 16 face Gauss points.
//
// One lane per (cell, conserved variable): 12 cells per wave, five lanes
// each (lanes 60-63 idle).  A cell's 34 x 5 coefficients do not fit one lane
// in FP64, and the weights are per variable (component-wise CWENOZ), so each
// lane runs the whole scheme for one variable; the five lanes of a cell load
// the same operator values (one request per cell, served by the same cache
// lines), and each gathers its own variable's row of the stencil states.
// Positivity needs all five variables of a point: the cell's lanes exchange
// them with ds_bpermute.

constexpr int kP4K = 34;        // basis terms of the degree-4 polynomial
constexpr int kP4KD = 9;        // basis terms of a quadratic directional polynomial
constexpr int kP4Cells = 12;    // cells per wave
constexpr int kP4Q = 16;        // Gauss points per quadrilateral face (4 x 4)
#ifndef P4_WAVES
#define P4_WAVES 2
#endif

// The 34 monomials of degree 1..4 in graded-lex order (x exponent
// descending, then y) at a face point's scaled offset, minus their cell
// means.
template <class T>
__device__ __forceinline__ void basis_p4(T x, T y, T z, const T* pm, T* ph) {
    const T xx = x * x, yy = y * y, zz = z * z;
    const T t[kP4K] = {x, y, z,
                       xx, x * y, x * z, yy, y * z, zz,
                       xx * x, xx * y, xx * z, x * yy, x * y * z, x * zz, yy * y, yy * z, y * zz, zz * z,
                       xx * xx, xx * x * y, xx * x * z, xx * yy, xx * y * z, xx * zz, x * yy * y, x * yy * z,
                       x * y * zz, x * zz * z, yy * yy, yy * y * z, yy * zz, y * zz * z, zz * zz};
#pragma unroll
    for (int k = 0; k < kP4K; ++k) ph[k] = t[k] - pm[k];
}

// value of x in lane src of the wave (per-lane source)
template <class T>
__device__ __forceinline__ T p4_from(T x, int src) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_ds_bpermute(src << 2, __builtin_bit_cast(int, x)));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, x);
        const uint32_t lo = uint32_t(__builtin_amdgcn_ds_bpermute(src << 2, int(uint32_t(u))));
        const uint32_t hi = uint32_t(__builtin_amdgcn_ds_bpermute(src << 2, int(uint32_t(u >> 32))));
        return __builtin_bit_cast(T, (uint64_t(hi) << 32) | lo);
    }
}

// Steps per lane (cell c, variable v):
//  (i)   jumps b_m = U_m,v - U_c,v in FP64, rounded to T
//  (ii)  a = B_c b (34 terms)
//  (iii) SI_1 = a^T O a
//  (iv)  per directional stencil s: a_s = B_s b_s (9 terms), SI_s = a_s^T O_9 a_s
//        with O_9 the block of O on the first 9 (degree <= 2) terms
//  (v)   tau = mean_s |SI_1 - SI_s|; LPR blend
//        abar = s1 a + (tau/W) G on the first 9 terms, s1 = (1 + tau/(eps+SI_1))/W,
//        W = 1 + tau sum_s lambda_s/(eps+SI_s), G = sum_s lambda_s (r_s - r_1) a_s
//  (vi)  point values U_c,v + Phi_q . abar; positivity of rho and p at each point.
// LABEL: also max over stencils and variables of |omega - lambda| per cell.
template <class T, bool LABEL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(P4_WAVES)))
void reconstruct_p4_kernel(ReconArgs<T> A) {
    constexpr int K = kP4K, KD = kP4KD;
    const int64_t nc = A.nc;
    const int lane = int(threadIdx.x & 63u);
    const int slot = lane / 5, v = lane - 5 * slot;
    const int64_t c0 = (xcd_block() * (kBlock / 64) + int64_t(threadIdx.x >> 6)) * kP4Cells;
    const bool valid = slot < kP4Cells && c0 + slot < nc;
    // idle lanes shadow the wave's first cell (every load stays in range)
    const int64_t c = valid ? c0 + slot : (c0 < nc ? c0 : nc - 1);
    const int vv = valid ? v : 0;
    const double ui = A.U[vv * nc + c];
    const double* Uv = A.U + int64_t(vv) * nc;

    // (ii) central coefficients; member m's id at sten_c[m][c], its K
    // operator rows at Bc[m][k][c].  Operators and states load one member
    // ahead of the arithmetic, ids two ahead (a state load waits only for an
    // id loaded an iteration earlier).
    T a[K];
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = T(0);
    const int MC = A.MC;
    {
        auto last = [&](int m) { return m < MC ? m : MC - 1; };
        double un = Uv[A.sten_c[c]];
        int32_t j2 = A.sten_c[int64_t(last(1)) * nc + c];
        T bn[K];
#pragma unroll
        for (int k = 0; k < K; ++k) bn[k] = A.Bc[int64_t(k) * nc + c];
#pragma unroll 1
        for (int m = 0; m < MC; ++m) {
            const T bv = T(un - ui);
            T b[K];
#pragma unroll
            for (int k = 0; k < K; ++k) b[k] = bn[k];
            const int mf = last(m + 1);
            un = Uv[j2];
            j2 = A.sten_c[int64_t(last(m + 2)) * nc + c];
#pragma unroll
            for (int k = 0; k < K; ++k) bn[k] = A.Bc[(int64_t(mf) * K + k) * nc + c];
#pragma unroll
            for (int k = 0; k < K; ++k) a[k] += b[k] * bv;
        }
    }

    // (iii) SI_1 = a^T O a, O as its upper triangle (sum of squares: a
    // rounded value below zero is clamped)
    T SI1 = T(0);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        T t = A.O[int64_t(tri_index(K, k, k)) * nc + c] * a[k];
#pragma unroll
        for (int l = k + 1; l < K; ++l) t += T(2) * A.O[int64_t(tri_index(K, k, l)) * nc + c] * a[l];
        SI1 += a[k] * t;
    }
    SI1 = fmax(SI1, T(0));

    // (iv) directional stencils
    const int nd = int(A.ndir[c]);
    const T lam_s = T(1) / (A.lam_c + T(nd > 0 ? nd : 1)), lam_1 = A.lam_c * lam_s;
    const T r1 = T(1) / (A.eps + SI1);
    T G[KD], tsum = T(0), Lam = lam_1 * r1;
    T rs[kMaxFaces];
#pragma unroll
    for (int k = 0; k < KD; ++k) G[k] = T(0);
#pragma unroll
    for (int s = 0; s < kMaxFaces; ++s) rs[s] = r1;
    if (nd > 0) {
        const int MD = A.MD;
#pragma unroll 1
        for (int s = 0; s < A.ND; ++s) {
            T as[KD];
#pragma unroll
            for (int k = 0; k < KD; ++k) as[k] = T(0);
            const int64_t r0 = int64_t(s) * MD;
            auto row = [&](int j) { return r0 + (j < MD ? j : MD - 1); };
            double un = Uv[A.sten_d[r0 * nc + c]];
            int32_t j2 = A.sten_d[row(1) * nc + c];
            T bn[KD];
#pragma unroll
            for (int k = 0; k < KD; ++k) bn[k] = A.Bd[(r0 * KD + k) * nc + c];
#pragma unroll 1
            for (int j = 0; j < MD; ++j) {
                const T bv = T(un - ui);
                T b[KD];
#pragma unroll
                for (int k = 0; k < KD; ++k) b[k] = bn[k];
                const int64_t rf = row(j + 1);
                un = Uv[j2];
                j2 = A.sten_d[row(j + 2) * nc + c];
#pragma unroll
                for (int k = 0; k < KD; ++k) bn[k] = A.Bd[(rf * KD + k) * nc + c];
#pragma unroll
                for (int k = 0; k < KD; ++k) as[k] += b[k] * bv;
            }
            if (s < nd) {
                // SI_s with the block of O on the first KD terms (its upper
                // triangle read per stencil: cache hits after the first)
                T SIs = T(0);
#pragma unroll
                for (int k = 0; k < KD; ++k) {
                    T t = A.O[int64_t(tri_index(K, k, k)) * nc + c] * as[k];
#pragma unroll
                    for (int l = k + 1; l < KD; ++l) t += T(2) * A.O[int64_t(tri_index(K, k, l)) * nc + c] * as[l];
                    SIs += as[k] * t;
                }
                SIs = fmax(SIs, T(0));
                tsum += fabs(SI1 - SIs);
                const T r = T(1) / (A.eps + SIs);
                Lam += lam_s * r;
#pragma unroll
                for (int t = 0; t < kMaxFaces; ++t)
                    if (t == s) rs[t] = r;
                const T coef = lam_s * (r - r1);
#pragma unroll
                for (int k = 0; k < KD; ++k) G[k] += coef * as[k];
            }
        }
    }
    // (v) blend
    float lab = 0.f;
    if (nd > 0) {
        const T tau = tsum / T(nd);
        const T W = T(1) + tau * Lam;
        const T s1 = (T(1) + tau * r1) / W;
        const T tw = tau / W;
#pragma unroll
        for (int k = 0; k < K; ++k) a[k] *= s1;
#pragma unroll
        for (int k = 0; k < KD; ++k) a[k] += tw * G[k];
        if constexpr (LABEL) {
            lab = float(fabs(lam_1 * (s1 - T(1))));
#pragma unroll
            for (int s = 0; s < kMaxFaces; ++s)
                if (s < nd) lab = fmaxf(lab, float(fabs(lam_s * ((T(1) + tau * rs[s]) / W - T(1)))));
        }
    }

    // (vi) point values at the cell's face points, slots [lf][q][v][cell]
    T pm[K];
#pragma unroll
    for (int k = 0; k < K; ++k) pm[k] = A.pmean[int64_t(k) * nc + c];
    const int base = slot < kP4Cells ? 5 * slot : 0;
    bool ok = true;
    const int NF = A.NF, Q = A.Q;
#pragma unroll 1
    for (int lf = 0; lf < NF; ++lf) {
        const int nq = A.cnq[int64_t(lf) * nc + c];
#pragma unroll 1
        for (int q = 0; q < Q; ++q) {
            if (q >= nq) break;  // uniform within a cell's five lanes
            const int64_t row = (int64_t(lf) * Q + q) * 3;
            const T x = A.xi[row * nc + c], y = A.xi[(row + 1) * nc + c], z = A.xi[(row + 2) * nc + c];
            T ph[K];
            basis_p4<T>(x, y, z, pm, ph);
            T d = T(0);
#pragma unroll
            for (int k = 0; k < K; ++k) d += ph[k] * a[k];
            const T val = T(ui + double(d));
            if (valid) A.fs[((int64_t(lf) * Q + q) * 5 + v) * nc + c] = val;
            // the point's five variables from the cell's lanes
            const T r = p4_from(val, base), mx = p4_from(val, base + 1), my = p4_from(val, base + 2),
                    mz = p4_from(val, base + 3), E = p4_from(val, base + 4);
            const T p = A.gm1 * (E - T(0.5) * (mx * mx + my * my + mz * mz) / r);
            ok = ok && (r > T(1e-10)) && (p > T(1e-10));
        }
    }
    if constexpr (LABEL) {
#pragma unroll
        for (int t = 1; t < 5; ++t) lab = fmaxf(lab, p4_from(lab, base + t));
    }
    if (valid && v == 0) {
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
            for (int v = 0; v < 5; ++v) A.fs[((int64_t(lf) * A.Q + q) * 5 + v) * nc + c] = T(A.U[v * nc + c]);
    }
    A.flags[c] = uint8_t((fl & 0x7f) | 4);
}
