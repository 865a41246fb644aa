// Troubled-cell gate network on CDNA4 matrix cores (included by
// ucns_kernels.hip).  12 -> 64 -> 64 -> 1, ReLU, sigmoid; BF16 operands with
// FP32 accumulation on v_mfma_f32_16x16x32_bf16.  Lane layout of that
// instruction (lane l, g = l / 16, r = l % 16):
//   A (16 x 32): row r, k = 8 g .. 8 g + 7      B (32 x 16): column r, same k
//   C (16 x 16): column r, rows 4 g .. 4 g + 3
// One wave evaluates 64 cells: their feature rows are staged in LDS and
// re-read as A fragments; the weights are staged once per block as bf16.
//
// Parameter block (float32, offsets below): mu[16] isig[16] W1[16][64] b1[64]
// W2[64][64] b2[64] w3[64] b3 theta.  W1[k][n] maps input k to hidden n.

typedef __bf16 ucns_bf16x8 __attribute__((ext_vector_type(8)));
typedef float ucns_f32x4 __attribute__((ext_vector_type(4)));

namespace mlp {
constexpr int kOffMu = 0, kOffIsig = 16, kOffW1 = 32, kOffB1 = 1056, kOffW2 = 1120, kOffB2 = 5216, kOffW3 = 5280,
              kOffB3 = 5344, kOffTheta = 5345, kNParam = 5348;
constexpr int kXS = 24;  // LDS row stride (bf16) of 16-wide rows: 48 B, keeps 16-B alignment
constexpr int kHS = 72;  // LDS row stride (bf16) of 64-wide rows: 144 B, staggers banks
}  // namespace mlp

// float -> bfloat16 bits, round to nearest with ties to even (inputs finite)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

__device__ __forceinline__ ucns_bf16x8 lds8(const uint16_t* p) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    return __builtin_bit_cast(ucns_bf16x8, v);
}

__device__ __forceinline__ ucns_f32x4 mfma16(ucns_bf16x8 a, ucns_bf16x8 b, ucns_f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ ucns_bf16x8 zero8() {
    const uint4 z = make_uint4(0, 0, 0, 0);
    return __builtin_bit_cast(ucns_bf16x8, z);
}

// Block-shared copy of the network (bf16 matrices, fp32 vectors).
struct MlpWeights {
    alignas(16) uint16_t W1t[64 * mlp::kXS];  // [n][k], k < 16
    alignas(16) uint16_t W2t[64 * mlp::kHS];  // [n_out][k_in]
    float b1[64], b2[64], w3[64], mu[16], isig[16];
    float b3, theta;
};

__device__ void mlp_stage(const float* __restrict__ P, MlpWeights& S, int tid, int nthr) {
    // consecutive threads read consecutive n (coalesced), write transposed to LDS
    for (int i = tid; i < 64 * 16; i += nthr) {
        const int k = i >> 6, n = i & 63;
        S.W1t[n * mlp::kXS + k] = f2bf(P[mlp::kOffW1 + k * 64 + n]);
    }
    for (int i = tid; i < 64 * 64; i += nthr) {
        const int k = i >> 6, n = i & 63;
        S.W2t[n * mlp::kHS + k] = f2bf(P[mlp::kOffW2 + k * 64 + n]);
    }
    for (int i = tid; i < 64; i += nthr) {
        S.b1[i] = P[mlp::kOffB1 + i];
        S.b2[i] = P[mlp::kOffB2 + i];
        S.w3[i] = P[mlp::kOffW3 + i];
    }
    for (int i = tid; i < 16; i += nthr) {
        S.mu[i] = P[mlp::kOffMu + i];
        S.isig[i] = P[mlp::kOffIsig + i];
    }
    if (tid == 0) {
        S.b3 = P[mlp::kOffB3];
        S.theta = P[mlp::kOffTheta];
    }
}

// Per-wave scratch: rows of 64 cells (the X rows share the H buffer's start).
struct MlpWaveLds {
    alignas(16) uint16_t H[64 * mlp::kHS];
};

// Standardised inputs x[16] of this lane's cell -> logit z.  All 64 lanes of
// the wave must call it together (lanes without a cell pass zeros).
//
// Both layers are computed transposed (weights as the A operand, the cells'
// rows as B), so that a lane's output fragment holds four consecutive hidden
// units of one cell: the hidden layer is stored with one 8-byte LDS write per
// tile, and the output row sum needs only the four lane groups (two
// shuffles), after which lane l holds cell l's sum.
__device__ float mlp_wave_forward(const MlpWeights& S, MlpWaveLds& W, const float* f12) {
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    uint16_t* X = W.H;  // 64 rows x kXS, overwritten by the first hidden layer below
    {
        uint32_t w[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float x0 = 2 * k < 12 ? (f12[2 * k] - S.mu[2 * k]) * S.isig[2 * k] : 0.f;
            const float x1 = 2 * k + 1 < 12 ? (f12[2 * k + 1] - S.mu[2 * k + 1]) * S.isig[2 * k + 1] : 0.f;
            w[k] = uint32_t(f2bf(x0)) | (uint32_t(f2bf(x1)) << 16);
        }
        uint4* xr = reinterpret_cast<uint4*>(&X[lane * mlp::kXS]);
        xr[0] = make_uint4(w[0], w[1], w[2], w[3]);
        xr[1] = make_uint4(w[4], w[5], w[6], w[7]);
    }
    __builtin_amdgcn_wave_barrier();
    ucns_bf16x8 bx[4];  // B fragments: cells 16 mt + r, inputs 8 g .. 8 g + 7
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) bx[mt] = g < 2 ? lds8(&X[(16 * mt + r) * mlp::kXS + 8 * g]) : zero8();
    // The X rows now sit in registers (bx); the wave's LDS operations run in
    // issue order, so the hidden layer may overwrite them tile by tile.
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const ucns_bf16x8 aw = g < 2 ? lds8(&S.W1t[(16 * nt + r) * mlp::kXS + 8 * g]) : zero8();
        const int n0 = 16 * nt + 4 * g;  // this lane's hidden units n0 .. n0 + 3
        float bias[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) bias[j] = S.b1[n0 + j];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const ucns_f32x4 h = mfma16(aw, bx[mt], ucns_f32x4{0.f, 0.f, 0.f, 0.f});
            const uint32_t lo = uint32_t(f2bf(fmaxf(h[0] + bias[0], 0.f))) |
                                (uint32_t(f2bf(fmaxf(h[1] + bias[1], 0.f))) << 16);
            const uint32_t hi = uint32_t(f2bf(fmaxf(h[2] + bias[2], 0.f))) |
                                (uint32_t(f2bf(fmaxf(h[3] + bias[3], 0.f))) << 16);
            *reinterpret_cast<uint2*>(&W.H[(16 * mt + r) * mlp::kHS + n0]) = make_uint2(lo, hi);
        }
    }
    __builtin_amdgcn_wave_barrier();
    ucns_bf16x8 bh0[4], bh1[4];  // B fragments: cells 16 mt + r, hidden 8 g .. and 32 + 8 g ..
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        bh0[mt] = lds8(&W.H[(16 * mt + r) * mlp::kHS + 8 * g]);
        bh1[mt] = lds8(&W.H[(16 * mt + r) * mlp::kHS + 32 + 8 * g]);
    }
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const ucns_bf16x8 a0 = lds8(&S.W2t[(16 * nt + r) * mlp::kHS + 8 * g]);
        const ucns_bf16x8 a1 = lds8(&S.W2t[(16 * nt + r) * mlp::kHS + 32 + 8 * g]);
        const int n0 = 16 * nt + 4 * g;
        float bias[4], w[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            bias[j] = S.b2[n0 + j];
            w[j] = S.w3[n0 + j];
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            ucns_f32x4 acc = mfma16(a0, bh0[mt], ucns_f32x4{0.f, 0.f, 0.f, 0.f});
            acc = mfma16(a1, bh1[mt], acc);
#pragma unroll
            for (int j = 0; j < 4; ++j) part[mt] += fmaxf(acc[j] + bias[j], 0.f) * w[j];
        }
    }
    // sum over the four lane groups (output units 4 g .. 4 g + 3 of each tile)
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        part[mt] += __shfl_xor(part[mt], 16);
        part[mt] += __shfl_xor(part[mt], 32);
    }
    // lane l = 16 g + r holds cell 16 mt + r in part[mt]; its own cell is mt = g
    const float z = g == 0 ? part[0] : g == 1 ? part[1] : g == 2 ? part[2] : part[3];
    return z + S.b3;
}

// ------------------------------------------------------------ packed image
//
// Bytes [0, 4096): layer-1 A fragments, (nt, lane) at 16 (64 nt + lane):
// W1t[16 nt + r][8 g .. 8 g + 7] (zero for g >= 2); [4096, 12288): layer-2
// A fragments, (nt, half, lane) at 4096 + 16 (64 (2 nt + half) + lane):
// W2t[16 nt + r][32 half + 8 g .. + 7]; then float32 mu[16] isig[16] b1[64]
// b2[64] w3[64] b3 theta.
namespace mlpimg {
constexpr int kW1 = 0, kW2 = 4096, kF = 12288;
constexpr int kMu = 0, kIsig = 16, kB1 = 32, kB2 = 96, kW3 = 160, kB3 = 224, kTheta = 225, kNF = 226;
}  // namespace mlpimg

__global__ __launch_bounds__(256) void mlp_pack_kernel(const float* __restrict__ P, unsigned char* img) {
    for (int fr = threadIdx.x; fr < 4 * 64 + 8 * 64; fr += blockDim.x) {
        const int lane = fr & 63, g = lane >> 4, r = lane & 15;
        uint32_t w[4];
        if (fr < 256) {  // layer 1
            const int nt = fr >> 6, n = 16 * nt + r;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k0 = 8 * g + 2 * i;
                const uint32_t lo = g < 2 ? f2bf(P[mlp::kOffW1 + k0 * 64 + n]) : 0u;
                const uint32_t hi = g < 2 ? f2bf(P[mlp::kOffW1 + (k0 + 1) * 64 + n]) : 0u;
                w[i] = lo | (hi << 16);
            }
            *reinterpret_cast<uint4*>(img + mlpimg::kW1 + 16 * fr) = make_uint4(w[0], w[1], w[2], w[3]);
        } else {  // layer 2
            const int q = (fr - 256) >> 6, nt = q >> 1, half = q & 1, n = 16 * nt + r;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k0 = 32 * half + 8 * g + 2 * i;
                const uint32_t lo = f2bf(P[mlp::kOffW2 + k0 * 64 + n]);
                const uint32_t hi = f2bf(P[mlp::kOffW2 + (k0 + 1) * 64 + n]);
                w[i] = lo | (hi << 16);
            }
            *reinterpret_cast<uint4*>(img + mlpimg::kW2 + 16 * (fr - 256)) = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
    float* fv = reinterpret_cast<float*>(img + mlpimg::kF);
    for (int i = threadIdx.x; i < mlpimg::kNF; i += blockDim.x) {
        float x;
        if (i < mlpimg::kIsig) x = P[mlp::kOffMu + i];
        else if (i < mlpimg::kB1) x = P[mlp::kOffIsig + i - mlpimg::kIsig];
        else if (i < mlpimg::kB2) x = P[mlp::kOffB1 + i - mlpimg::kB1];
        else if (i < mlpimg::kW3) x = P[mlp::kOffB2 + i - mlpimg::kB2];
        else if (i < mlpimg::kB3) x = P[mlp::kOffW3 + i - mlpimg::kW3];
        else if (i == mlpimg::kB3) x = P[mlp::kOffB3];
        else x = P[mlp::kOffTheta];
        fv[i] = x;
    }
}

__device__ __forceinline__ ucns_bf16x8 gld8(const unsigned char* p) {
    return __builtin_bit_cast(ucns_bf16x8, *reinterpret_cast<const uint4*>(p));
}

// As mlp_wave_forward, with the weights read from the packed image (each
// lane loads its own 16-byte fragments; the vectors are small, cached reads).
__device__ float mlp_wave_forward_packed(const unsigned char* __restrict__ img, MlpWaveLds& W, const float* f12) {
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const float* fv = reinterpret_cast<const float*>(img + mlpimg::kF);
    uint16_t* X = W.H;
    {
        uint32_t w[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int k0 = 2 * k, k1 = 2 * k + 1;
            const float x0 = k0 < 12 ? (f12[k0] - fv[mlpimg::kMu + k0]) * fv[mlpimg::kIsig + k0] : 0.f;
            const float x1 = k1 < 12 ? (f12[k1] - fv[mlpimg::kMu + k1]) * fv[mlpimg::kIsig + k1] : 0.f;
            w[k] = uint32_t(f2bf(x0)) | (uint32_t(f2bf(x1)) << 16);
        }
        uint4* xr = reinterpret_cast<uint4*>(&X[lane * mlp::kXS]);
        xr[0] = make_uint4(w[0], w[1], w[2], w[3]);
        xr[1] = make_uint4(w[4], w[5], w[6], w[7]);
    }
    ucns_bf16x8 aw[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) aw[nt] = gld8(img + mlpimg::kW1 + 16 * (64 * nt + lane));
    __builtin_amdgcn_wave_barrier();
    ucns_bf16x8 bx[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) bx[mt] = g < 2 ? lds8(&X[(16 * mt + r) * mlp::kXS + 8 * g]) : zero8();
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int n0 = 16 * nt + 4 * g;
        const float4 bias = *reinterpret_cast<const float4*>(fv + mlpimg::kB1 + n0);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const ucns_f32x4 h = mfma16(aw[nt], bx[mt], ucns_f32x4{0.f, 0.f, 0.f, 0.f});
            const uint32_t lo = uint32_t(f2bf(fmaxf(h[0] + bias.x, 0.f))) |
                                (uint32_t(f2bf(fmaxf(h[1] + bias.y, 0.f))) << 16);
            const uint32_t hi = uint32_t(f2bf(fmaxf(h[2] + bias.z, 0.f))) |
                                (uint32_t(f2bf(fmaxf(h[3] + bias.w, 0.f))) << 16);
            *reinterpret_cast<uint2*>(&W.H[(16 * mt + r) * mlp::kHS + n0]) = make_uint2(lo, hi);
        }
    }
    __builtin_amdgcn_wave_barrier();
    ucns_bf16x8 bh0[4], bh1[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        bh0[mt] = lds8(&W.H[(16 * mt + r) * mlp::kHS + 8 * g]);
        bh1[mt] = lds8(&W.H[(16 * mt + r) * mlp::kHS + 32 + 8 * g]);
    }
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const ucns_bf16x8 a0 = gld8(img + mlpimg::kW2 + 16 * (64 * (2 * nt) + lane));
        const ucns_bf16x8 a1 = gld8(img + mlpimg::kW2 + 16 * (64 * (2 * nt + 1) + lane));
        const int n0 = 16 * nt + 4 * g;
        const float4 bias = *reinterpret_cast<const float4*>(fv + mlpimg::kB2 + n0);
        const float4 w = *reinterpret_cast<const float4*>(fv + mlpimg::kW3 + n0);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            ucns_f32x4 acc = mfma16(a0, bh0[mt], ucns_f32x4{0.f, 0.f, 0.f, 0.f});
            acc = mfma16(a1, bh1[mt], acc);
            // same summation order as mlp_wave_forward (identical decisions)
            part[mt] += fmaxf(acc[0] + bias.x, 0.f) * w.x;
            part[mt] += fmaxf(acc[1] + bias.y, 0.f) * w.y;
            part[mt] += fmaxf(acc[2] + bias.z, 0.f) * w.z;
            part[mt] += fmaxf(acc[3] + bias.w, 0.f) * w.w;
        }
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        part[mt] += __shfl_xor(part[mt], 16);
        part[mt] += __shfl_xor(part[mt], 32);
    }
    const float z = g == 0 ? part[0] : g == 1 ? part[1] : g == 2 ? part[2] : part[3];
    return z + fv[mlpimg::kB3];
}

// prob[i] = sigmoid(z) (mode 0) or mask[i] = sigmoid(z) < theta (mode 1)
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ P, const float* __restrict__ feat,
                                                          int64_t n, float* prob, uint8_t* mask) {
    __shared__ MlpWeights S;
    __shared__ MlpWaveLds Wv[4];
    mlp_stage(P, S, threadIdx.x, blockDim.x);
    __syncthreads();
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    float f[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) f[k] = i < n ? feat[i * 12 + k] : S.mu[k];
    const float z = mlp_wave_forward(S, Wv[threadIdx.x >> 6], f);
    if (i < n) {
        const float p = 1.f / (1.f + __expf(-z));
        if (prob) prob[i] = p;
        if (mask) mask[i] = p < S.theta ? 1 : 0;
    }
}

// ----------------------------------------------------------------- training
//
// The batch is cut into chunks of 64 samples (lane = sample); block b (one
// wave) takes chunks b, b + nblk, ... and writes its gradient partial:
//   x = bf16((f - mu) isig); H1 = relu(x W1 + b1); H2 = relu(bf16(H1) W2 + b2)
//   z = H2 . w3 + b3; loss = mean_w BCE(z, y); dz = w (sigmoid(z) - y) / B
//   dH2 = dz w3 [H2 > 0]; dW2 = bf16(H1)^T bf16(dH2); dw3 = H2^T dz
//   dH1 = bf16(dH2) W2^T [H1 > 0]; dW1 = x^T bf16(dH1); db = column sums
// mlp_adam_kernel then sums the partials in block order (the result depends
// on n only, not on scheduling) and applies Adam (FP32 master weights) on the
// trainable slots.
namespace mlp {
constexpr int kTrainMaxBlocks = 64;
constexpr int kTrainStride = 5376;  // floats per partial row: kNParam slots, then the loss
}  // namespace mlp
struct TrainLds {
    MlpWeights S;
    uint16_t W2r[64 * mlp::kHS];   // [k_in][n_out] (row-major W2) for dH1
    uint16_t Xs[64 * mlp::kXS];    // [r][k]
    uint16_t Xt[16 * mlp::kHS];    // [k][r]
    uint16_t Hs[64 * mlp::kHS];    // bf16(H1) [r][i]
    uint16_t H1t[64 * mlp::kHS];   // [i][r]; later dH1 [i][r]
    uint16_t dH2s[64 * mlp::kHS];  // [r][n]
    uint16_t dH2t[64 * mlp::kHS];  // [n][r]
    float z[64], dz[64];
    float red[64];
};

__global__ __launch_bounds__(64) void mlp_train_kernel(const float* __restrict__ P, float* __restrict__ part,
                                                       const float* __restrict__ feat, const float* __restrict__ lab,
                                                       int64_t n, float pos_w) {
    __shared__ TrainLds L;
    const int lane = threadIdx.x, g = lane >> 4, r = lane & 15;
    mlp_stage(P, L.S, lane, 64);
    for (int i = lane; i < 64 * 64; i += 64) {
        const int k = i >> 6, nn = i & 63;
        L.W2r[k * mlp::kHS + nn] = f2bf(P[mlp::kOffW2 + k * 64 + nn]);
    }
    __syncthreads();
    const MlpWeights& S = L.S;
    // gradient accumulators: dW1 tile (k, n) for nt; dW2 tiles (it, nt); per-lane column sums
    ucns_f32x4 gW1[4], gW2[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW1[a] = ucns_f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 4; ++b) gW2[a][b] = ucns_f32x4{0.f, 0.f, 0.f, 0.f};
    }
    float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, lsum = 0.f;  // lane = column index
    const float inv_b = 1.f / float(n);
    const int64_t nch = (n + 63) / 64;
    for (int64_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
        const int64_t i = ch * 64 + lane;
        const bool valid = i < n;
        // ---- inputs
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const float x = (k < 12 && valid) ? (feat[i * 12 + k] - S.mu[k]) * S.isig[k] : 0.f;
            const uint16_t xb = f2bf(x);
            L.Xs[lane * mlp::kXS + k] = xb;
            L.Xt[k * mlp::kHS + lane] = xb;
        }
        const float y = valid ? lab[i] : 0.f;
        const float wcls = valid ? (y > 0.5f ? pos_w : 1.f) : 0.f;
        __builtin_amdgcn_wave_barrier();
        // ---- layer 1
        ucns_bf16x8 ax[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) ax[mt] = g < 2 ? lds8(&L.Xs[(16 * mt + r) * mlp::kXS + 8 * g]) : zero8();
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const ucns_bf16x8 bw = g < 2 ? lds8(&S.W1t[(16 * nt + r) * mlp::kXS + 8 * g]) : zero8();
            const int nn = 16 * nt + r;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const ucns_f32x4 acc = mfma16(ax[mt], bw, ucns_f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint16_t hb = f2bf(fmaxf(acc[j] + S.b1[nn], 0.f));
                    const int row = 16 * mt + 4 * g + j;
                    L.Hs[row * mlp::kHS + nn] = hb;
                    L.H1t[nn * mlp::kHS + row] = hb;
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        // ---- layer 2, pass A: logits
        float part[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) part[mt][j] = 0.f;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const ucns_bf16x8 b0 = lds8(&S.W2t[(16 * nt + r) * mlp::kHS + 8 * g]);
            const ucns_bf16x8 b1 = lds8(&S.W2t[(16 * nt + r) * mlp::kHS + 32 + 8 * g]);
            const int nn = 16 * nt + r;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                ucns_f32x4 acc = mfma16(lds8(&L.Hs[(16 * mt + r) * mlp::kHS + 8 * g]), b0, ucns_f32x4{0.f, 0.f, 0.f, 0.f});
                acc = mfma16(lds8(&L.Hs[(16 * mt + r) * mlp::kHS + 32 + 8 * g]), b1, acc);
#pragma unroll
                for (int j = 0; j < 4; ++j) part[mt][j] += fmaxf(acc[j] + S.b2[nn], 0.f) * S.w3[nn];
            }
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float v = part[mt][j];
                v += __shfl_xor(v, 1, 16);
                v += __shfl_xor(v, 2, 16);
                v += __shfl_xor(v, 4, 16);
                v += __shfl_xor(v, 8, 16);
                if (r == 0) L.z[16 * mt + 4 * g + j] = v + S.b3;
            }
        __builtin_amdgcn_wave_barrier();
        {
            const float z = L.z[lane];
            const float s = 1.f / (1.f + __expf(-z));
            const float d = wcls * (s - y) * inv_b;
            L.dz[lane] = d;
            // BCE with logits: log(1 + e^-|z|) + max(z, 0) - z y
            lsum += wcls * (log1pf(__expf(-fabsf(z))) + fmaxf(z, 0.f) - z * y);
            gb3 += d;
        }
        __builtin_amdgcn_wave_barrier();
        // ---- layer 2, pass B: dH2, dw3, db2 (recomputing H2 from the same products)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const ucns_bf16x8 b0 = lds8(&S.W2t[(16 * nt + r) * mlp::kHS + 8 * g]);
            const ucns_bf16x8 b1 = lds8(&S.W2t[(16 * nt + r) * mlp::kHS + 32 + 8 * g]);
            const int nn = 16 * nt + r;
            float cw3 = 0.f, cb2 = 0.f;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                ucns_f32x4 acc = mfma16(lds8(&L.Hs[(16 * mt + r) * mlp::kHS + 8 * g]), b0, ucns_f32x4{0.f, 0.f, 0.f, 0.f});
                acc = mfma16(lds8(&L.Hs[(16 * mt + r) * mlp::kHS + 32 + 8 * g]), b1, acc);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = 16 * mt + 4 * g + j;
                    const float h2p = acc[j] + S.b2[nn];
                    const float dzr = L.dz[row];
                    const float dh2 = h2p > 0.f ? dzr * S.w3[nn] : 0.f;
                    cw3 += fmaxf(h2p, 0.f) * dzr;
                    cb2 += dh2;
                    const uint16_t db = f2bf(dh2);
                    L.dH2s[row * mlp::kHS + nn] = db;
                    L.dH2t[nn * mlp::kHS + row] = db;
                }
            }
            // sum the column's partials over the 4 lane groups
            cw3 += __shfl_xor(cw3, 16);
            cw3 += __shfl_xor(cw3, 32);
            cb2 += __shfl_xor(cb2, 16);
            cb2 += __shfl_xor(cb2, 32);
            if (g == nt) {  // lane 16 nt + r keeps column nn = lane
                gw3 += cw3;
                gb2 += cb2;
            }
        }
        __builtin_amdgcn_wave_barrier();
        // ---- dW2[i][n] += sum_r H1[r][i] dH2[r][n]   (K = 64 samples = 2 steps)
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const ucns_bf16x8 a0 = lds8(&L.H1t[(16 * it + r) * mlp::kHS + 8 * g]);
            const ucns_bf16x8 a1 = lds8(&L.H1t[(16 * it + r) * mlp::kHS + 32 + 8 * g]);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                gW2[it][nt] = mfma16(a0, lds8(&L.dH2t[(16 * nt + r) * mlp::kHS + 8 * g]), gW2[it][nt]);
                gW2[it][nt] = mfma16(a1, lds8(&L.dH2t[(16 * nt + r) * mlp::kHS + 32 + 8 * g]), gW2[it][nt]);
            }
        }
        __builtin_amdgcn_wave_barrier();
        // ---- dH1[r][i] = sum_n dH2[r][n] W2[i][n] [H1 > 0]; written as [i][r] over H1t
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const ucns_bf16x8 b0 = lds8(&L.W2r[(16 * it + r) * mlp::kHS + 8 * g]);
            const ucns_bf16x8 b1 = lds8(&L.W2r[(16 * it + r) * mlp::kHS + 32 + 8 * g]);
            const int ii = 16 * it + r;
            float cb1 = 0.f;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                ucns_f32x4 acc = mfma16(lds8(&L.dH2s[(16 * mt + r) * mlp::kHS + 8 * g]), b0, ucns_f32x4{0.f, 0.f, 0.f, 0.f});
                acc = mfma16(lds8(&L.dH2s[(16 * mt + r) * mlp::kHS + 32 + 8 * g]), b1, acc);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = 16 * mt + 4 * g + j;
                    const float dh1 = (L.Hs[row * mlp::kHS + ii] & 0x7FFF) != 0 ? acc[j] : 0.f;
                    cb1 += dh1;
                    L.H1t[ii * mlp::kHS + row] = f2bf(dh1);
                }
            }
            cb1 += __shfl_xor(cb1, 16);
            cb1 += __shfl_xor(cb1, 32);
            if (g == it) gb1 += cb1;
        }
        __builtin_amdgcn_wave_barrier();
        // ---- dW1[k][i] += sum_r x[r][k] dH1[r][i]  (M = 16 inputs)
        {
            const ucns_bf16x8 a0 = lds8(&L.Xt[r * mlp::kHS + 8 * g]);
            const ucns_bf16x8 a1 = lds8(&L.Xt[r * mlp::kHS + 32 + 8 * g]);
#pragma unroll
            for (int it = 0; it < 4; ++it) {
                gW1[it] = mfma16(a0, lds8(&L.H1t[(16 * it + r) * mlp::kHS + 8 * g]), gW1[it]);
                gW1[it] = mfma16(a1, lds8(&L.H1t[(16 * it + r) * mlp::kHS + 32 + 8 * g]), gW1[it]);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    // ---- this block's partial (parameter layout; every trainable slot written)
    float* G = part + int64_t(blockIdx.x) * mlp::kTrainStride;
#pragma unroll
    for (int it = 0; it < 4; ++it)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * g + j;  // input row of W1 (rows 12..15 are padding)
            G[mlp::kOffW1 + k * 64 + 16 * it + r] = k < 12 ? gW1[it][j] : 0.f;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) G[mlp::kOffW2 + (16 * it + 4 * g + j) * 64 + 16 * nt + r] = gW2[it][nt][j];
        }
    G[mlp::kOffB1 + lane] = gb1;
    G[mlp::kOffB2 + lane] = gb2;
    G[mlp::kOffW3 + lane] = gw3;
    // wave sums of gb3 (per-sample dz) and the loss
    float s3 = gb3, sl = lsum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        s3 += __shfl_xor(s3, o);
        sl += __shfl_xor(sl, o);
    }
    if (lane == 0) {
        G[mlp::kOffB3] = s3;
        G[mlp::kNParam] = sl;
    }
}

// Sums the nblk partials of mlp_train_kernel in block order into G (zero on
// the untrained slots) and the mean loss, then one Adam step on [W1 .. b3].
__global__ __launch_bounds__(256) void mlp_adam_kernel(float* __restrict__ P, float* __restrict__ G,
                                                       float* __restrict__ Am, float* __restrict__ Av,
                                                       const float* __restrict__ part, int nblk, float inv_b, float lr,
                                                       int t, float* loss_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == mlp::kNParam) {
        float sl = 0.f;
        for (int b = 0; b < nblk; ++b) sl += part[int64_t(b) * mlp::kTrainStride + mlp::kNParam];
        if (loss_out) *loss_out = sl * inv_b;
        return;
    }
    if (i > mlp::kNParam) return;
    if (i < mlp::kOffW1 || i >= mlp::kOffTheta) {
        G[i] = 0.f;
        return;
    }
    float gi = 0.f;
    for (int b = 0; b < nblk; ++b) gi += part[int64_t(b) * mlp::kTrainStride + i];
    G[i] = gi;
    const float b1c = 1.f - powf(0.9f, float(t)), b2c = 1.f - powf(0.999f, float(t));
    const float m = 0.9f * Am[i] + 0.1f * gi;
    const float v = 0.999f * Av[i] + 0.001f * gi * gi;
    Am[i] = m;
    Av[i] = v;
    P[i] -= lr * (m / b1c) / (sqrtf(v / b2c) + 1e-8f);
}
