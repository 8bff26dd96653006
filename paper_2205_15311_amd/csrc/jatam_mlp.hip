// jatam_mlp.hip - the surrogate MLP: training and inference on gfx950.
//
// Not from the paper (which has no learned part): the surrogate predicts a
// genotype's class (UNBOUND / ND / DET) and log(1 + size) from its edge
// colours, so the batched path can order work and the GA can screen
// offspring; every reported class still comes from exact assembly.
//
// x = one-hot of the 12 edge colours (12 x 8; absent tiles all zero)
// h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2) (256 wide), out = h2 W3 + b3.
// Loss = mean cross-entropy of the 3 class logits + mean squared error of
// log1p(size).  Weights are kept in fp32 (with Adam moments) and used as
// bf16; h1, h2 and the hidden gradients are stored as bf16; every product
// accumulates in fp32.
//
//   layer 1      a gather: the sum of 4t rows of W1 (a one-hot input times a
//                matrix is no work for a matrix core)
//   h1 W2, dh2 W2^T, h1^T dh2, x^T dh1
//                bf16 MFMA GEMMs (v_mfma_f32_16x16x32_bf16), one wave per
//                16 x 16 output tile, fused bias/ReLU/mask epilogues
//   head, loss   per-sample dot products of length 256 and a softmax
//   Adam         elementwise over the 91,652 fp32 parameters
#include "jatam_device.hpp"
#include "jatam_internal.hpp"

namespace jatam {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

// fp32 -> bf16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t bf16_bits(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u)
        return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float bf16_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Keeps the bf16 copy of weight i (flat index) equal to its fp32 master.
// Also keeps the transposed copies the fused scoring kernel reads with k
// contiguous: w2t[n][k] = W2[k][n] and w3t[k][j] = W3[j][k] (rows 4..15 of
// w3t stay zero).
__device__ __forceinline__ void refresh_bf16(const MlpArgs& a, int i, float w)
{
    const uint16_t b = bf16_bits(w);
    if (i < kMlpOffB1) {
        a.w1b[i] = b;
    } else if (i >= kMlpOffW2 && i < kMlpOffB2) {
        const int r = i - kMlpOffW2;
        a.w2b[r] = b;
        a.w2t[(r % kMlpHidden) * kMlpHidden + r / kMlpHidden] = b;
    } else if (i >= kMlpOffW3 && i < kMlpOffB3) {
        const int r = i - kMlpOffW3;
        a.w3b[r] = b;
        a.w3t[(r % kMlpOut) * kMlpHidden + r / kMlpOut] = b;
    }
}

// Tiles the network reads of a genome of t tiles: the input has 12 edge slots
// (3 tiles), so a t outside 1..3 is read as no tiles at all (zero input).
__device__ __forceinline__ int mlp_tiles(int t) { return t >= 1 && t <= 3 ? t : 0; }

// ---------------------------------------------------------------------------
// Layer 1: h1 = bf16(relu(sum of W1 rows + b1)); also the one-hot x (bf16).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mlp_layer1_kernel(MlpArgs a, const uint64_t* genomes,
                                                         const uint8_t* tvec, int t_all,
                                                         uint32_t n)
{
    const uint32_t b = blockIdx.x;          // sample (rows n..gridDim.x-1 are padding)
    const int j = threadIdx.x;              // hidden unit
    if (b >= n) {
        a.h1[(size_t)b * kMlpHidden + j] = 0;
        if (j < kMlpIn)
            a.x[(size_t)b * kMlpIn + j] = 0;
        return;
    }
    const uint64_t g = genomes[b];
    const int t = mlp_tiles(tvec != nullptr ? tvec[b] : t_all);
    const uint32_t cmask = (uint32_t)a.c - 1u;
    float acc = 0.f;
    for (int e = 0; e < kMlpEdges; ++e) {
        if (e >= 4 * t)
            break;
        const uint32_t colour = (uint32_t)(g >> (a.bits * (4 * t - 1 - e))) & cmask;
        acc += bf16_float(a.w1b[(e * 8 + colour) * kMlpHidden + j]);
    }
    acc += a.p.b1[j];
    a.h1[(size_t)b * kMlpHidden + j] = bf16_bits(acc > 0.f ? acc : 0.f);   // +0, never -0
    if (j < kMlpIn) {
        const int e = j >> 3;
        uint32_t hot = 0;
        if (e < 4 * t)
            hot = ((uint32_t)(g >> (a.bits * (4 * t - 1 - e))) & cmask) == (uint32_t)(j & 7);
        a.x[(size_t)b * kMlpIn + j] = hot ? (uint16_t)0x3F80u : (uint16_t)0;   // 1.0 or 0.0
    }
}

// ---------------------------------------------------------------------------
// GEMM: C[M x N] = sum_k A(m, k) B(k, n), bf16 operands addressed by strides
// (so transposes cost nothing), fp32 accumulation in v_mfma_f32_16x16x32_bf16.
// One wave computes one 16 x 16 tile; K is a multiple of 32.
//
// Operand layout of the 16x16x32 MFMA (one wave): lane l holds
//   A[l % 16][8 * (l / 16) + i], i < 8      (16 x 32, M x K)
//   B[8 * (l / 16) + i][l % 16], i < 8      (32 x 16, K x N)
// and receives D[4 * (l / 16) + i][l % 16], i < 4.
// ---------------------------------------------------------------------------
enum { kEpStoreF32 = 0, kEpBiasRelu = 1, kEpReluMask = 2 };

struct GemmArgs {
    const uint16_t* A;
    int64_t sam, sak;        // A(m, k) = A[m * sam + k * sak]
    const uint16_t* B;
    int64_t sbk, sbn;        // B(k, n) = B[k * sbk + n * sbn]
    int M, N, K;
    int epilogue;
    float* C32;              // kEpStoreF32: C[m * N + n]
    uint16_t* C16;           // kEpBiasRelu / kEpReluMask: bf16 C[m * N + n]
    const float* bias;       // kEpBiasRelu: bias[n]
    const uint16_t* mask;    // kEpReluMask: keep where mask[m * N + n] > 0
    int splits;              // K split across this many workgroups (kEpStoreF32 only)
    float* partial;          // splits > 1: [splits][M][N] fp32 partial sums
};

__device__ __forceinline__ int lane16() { return (int)(__lane_id() & 15); }
__device__ __forceinline__ int quad() { return (int)(__lane_id() >> 4); }

// Block tile of the GEMM: 64 x 64 outputs per workgroup of 4 waves, each
// wave a 32 x 32 quarter (2 x 2 MFMA tiles), K in steps of 32.  Both operand
// tiles are staged in LDS with k contiguous, so every MFMA fragment is one
// 16-byte LDS read; the global loads are 16 bytes along whichever of the two
// dimensions is contiguous in memory (a transposed operand is scattered into
// LDS).  With splits > 1 the K range is split across workgroups and each
// writes fp32 partial sums, added in split order by mlp_reduce_kernel.
constexpr int kBM = 64, kBN = 64, kBK = 32, kLdsPitch = kBK + 8;

// One 64 x 32 operand tile into LDS (rows r0.., k k0..): element (r, k) of
// the operand is src[r * s_row + k * s_k]; rows >= R are zero.  Needs R a
// multiple of 8 and, for s_k != 1, s_row == 1.
__device__ __forceinline__ void load_tile(const uint16_t* __restrict__ src, int64_t s_row,
                                          int64_t s_k, int r0, int k0, int R,
                                          uint16_t (*dst)[kLdsPitch])
{
    const int tid = (int)threadIdx.x;
    if (s_k == 1) {
        const int r = tid >> 2, kc = (tid & 3) * 8;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (r0 + r < R)
            v = *reinterpret_cast<const uint4*>(src + (int64_t)(r0 + r) * s_row + k0 + kc);
        *reinterpret_cast<uint4*>(&dst[r][kc]) = v;
    } else {
        const int k = tid >> 3, rc = (tid & 7) * 8;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (r0 + rc < R)
            v = *reinterpret_cast<const uint4*>(src + (int64_t)(k0 + k) * s_k + r0 + rc);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 8; ++e)
            dst[rc + e][k] = (uint16_t)(w[e >> 1] >> (16 * (e & 1)));
    }
}

__global__ __launch_bounds__(256) void mlp_gemm_kernel(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[kBM][kLdsPitch];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kBN][kLdsPitch];
    const int wave = (int)(threadIdx.x >> 6), l = (int)(threadIdx.x & 63);
    const int tiles_n = (g.N + kBN - 1) / kBN;
    const int m0 = ((int)blockIdx.x / tiles_n) * kBM, n0 = ((int)blockIdx.x % tiles_n) * kBN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int split = (int)blockIdx.y;
    const int kper = ((g.K / kBK + g.splits - 1) / g.splits) * kBK;
    const int kbeg = split * kper, kend = min(g.K, kbeg + kper);
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kbeg; k0 < kend; k0 += kBK) {
        load_tile(g.A, g.sam, g.sak, m0, k0, g.M, As);
        load_tile(g.B, g.sbn, g.sbk, n0, k0, g.N, Bs);
        __syncthreads();
        bf16x8 af[2], bf[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            af[i] = *reinterpret_cast<const bf16x8*>(&As[wm + 16 * i + (l & 15)][8 * (l >> 4)]);
            bf[i] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 16 * i + (l & 15)][8 * (l >> 4)]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0,
                                                                     0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wm + 16 * i + 4 * (l >> 4) + e;
                const int n = n0 + wn + 16 * j + (l & 15);
                if (m >= g.M || n >= g.N)
                    continue;
                const float v = acc[i][j][e];
                const int64_t o = (int64_t)m * g.N + n;
                if (g.splits > 1) {
                    g.partial[(int64_t)split * g.M * g.N + o] = v;
                } else if (g.epilogue == kEpStoreF32) {
                    g.C32[o] = v;
                } else if (g.epilogue == kEpBiasRelu) {
                    const float z = v + g.bias[n];
                    g.C16[o] = bf16_bits(z > 0.f ? z : 0.f);
                } else {
                    g.C16[o] = bf16_bits(g.mask[o] != 0 ? v : 0.f);
                }
            }
        }
    }
}

// out[i] = sum over s < parts of partial[s * count + i], in that order.
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* __restrict__ partial,
                                                         int parts, int64_t count, float* out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count)
        return;
    float s = 0.f;
    for (int p = 0; p < parts; ++p)
        s += partial[(int64_t)p * count + i];
    out[i] = s;
}

// ---------------------------------------------------------------------------
// Fused scoring: 64 samples per workgroup in one pass.  The layer-1 gather
// writes h1 (bf16) to LDS; h1 W2 runs on the matrix cores, each wave taking
// 64 columns of all 64 rows (4 x 4 MFMA tiles, W2 read k-contiguous from its
// transposed copy); bias, ReLU and bf16 rounding give h2, which overwrites h1
// in LDS; the head h2 W3 is one more MFMA tile per wave (W3 padded to 16
// columns); then softmax and the score.  Same rounding points as the
// separate kernels (h1, h2 in bf16; fp32 sums).
// ---------------------------------------------------------------------------
constexpr int kScoreRows = 64;
constexpr int kH1Pitch = kMlpHidden + 8;

__global__ __launch_bounds__(256) void mlp_score_kernel(MlpArgs a, const uint64_t* genomes,
                                                        const uint8_t* tvec, int t_all,
                                                        uint32_t n, float* scores)
{
    __shared__ __attribute__((aligned(16))) uint16_t hs[kScoreRows][kH1Pitch];
    __shared__ float head[kScoreRows][kMlpOut];
    const int tid = (int)threadIdx.x, wave = tid >> 6, l = tid & 63;
    const uint32_t s0 = blockIdx.x * kScoreRows;
    const uint32_t cmask = (uint32_t)a.c - 1u;
    // layer 1: 8 columns of 8 samples per thread
    {
        const int c8 = (tid & 31) * 8;
        float b1v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            b1v[q] = a.p.b1[c8 + q];
        for (int i = 0; i < 8; ++i) {
            const int row = (tid >> 5) + 8 * i;
            const uint32_t sidx = s0 + (uint32_t)row;
            uint32_t packed[4] = {0u, 0u, 0u, 0u};
            if (sidx < n) {
                const uint64_t g = genomes[sidx];
                const int t = mlp_tiles(tvec != nullptr ? tvec[sidx] : t_all);
                float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                for (int e = 0; e < 4 * t; ++e) {
                    const uint32_t colour =
                        (uint32_t)(g >> (a.bits * (4 * t - 1 - e))) & cmask;
                    const uint4 w = *reinterpret_cast<const uint4*>(
                        a.w1b + (size_t)(e * 8 + colour) * kMlpHidden + c8);
                    const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        acc[q] += bf16_float((uint16_t)(ww[q >> 1] >> (16 * (q & 1))));
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const float v = acc[q] + b1v[q];
                    packed[q >> 1] |= (uint32_t)bf16_bits(v > 0.f ? v : 0.f) << (16 * (q & 1));
                }
            }
            *reinterpret_cast<uint4*>(&hs[row][c8]) =
                make_uint4(packed[0], packed[1], packed[2], packed[3]);
        }
    }
    __syncthreads();
    // h1 W2
    const int n0 = 64 * wave;
    floatx4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < kMlpHidden; k0 += 32) {
        bf16x8 af[4], bfr[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            af[i] = *reinterpret_cast<const bf16x8*>(&hs[16 * i + (l & 15)][k0 + 8 * (l >> 4)]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            bfr[j] = *reinterpret_cast<const bf16x8*>(
                a.w2t + (size_t)(n0 + 16 * j + (l & 15)) * kMlpHidden + k0 + 8 * (l >> 4));
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0,
                                                                     0, 0);
    }
    __syncthreads();   // every wave has read h1
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = n0 + 16 * j + (l & 15);
        const float b2 = a.p.b2[col];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float z = acc[i][j][e] + b2;
                hs[16 * i + 4 * (l >> 4) + e][col] = bf16_bits(z > 0.f ? z : 0.f);
            }
    }
    __syncthreads();
    // head: wave w takes rows 16w..16w+15
    floatx4 o = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < kMlpHidden; k0 += 32) {
        const bf16x8 af =
            *reinterpret_cast<const bf16x8*>(&hs[16 * wave + (l & 15)][k0 + 8 * (l >> 4)]);
        const bf16x8 bfr = *reinterpret_cast<const bf16x8*>(
            a.w3t + (size_t)(l & 15) * kMlpHidden + k0 + 8 * (l >> 4));
        o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr, o, 0, 0, 0);
    }
    if ((l & 15) < kMlpOut) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            head[16 * wave + 4 * (l >> 4) + e][l & 15] = o[e] + a.p.b3[l & 15];
    }
    __syncthreads();
    if (tid < kScoreRows && s0 + (uint32_t)tid < n) {
        const float o0 = head[tid][0], o1 = head[tid][1], o2 = head[tid][2], o3 = head[tid][3];
        // expected size of a deterministic structure: P(DET) e^pred - 1
        const float mx = fmaxf(o0, fmaxf(o1, o2));
        const float e0 = expf(o0 - mx), e1 = expf(o1 - mx), e2 = expf(o2 - mx);
        scores[s0 + tid] = e2 / (e0 + e1 + e2) * expf(o3) - 1.f;
    }
}

// ---------------------------------------------------------------------------
// Persistent scoring: eight waves per workgroup, wave w owning hidden columns
// 32w .. 32w+31 of both layers.  Its slices of W1, W2 and W3 are loaded into
// registers once per launch as MFMA B operands, so a tile of 64 genomes
// costs no weight traffic at all:
//   layer 1   the one-hot input is a matrix like any other: each lane builds
//             its A operand (8 bf16 of one edge's one-hot row) from the
//             genome in registers, x W1 in v_mfma_f32_16x16x32_bf16 (2 k
//             blocks for two-tile genomes, 3 for three), + b1, ReLU, bf16
//             -> h1 in LDS (the wave's 32 columns)
//   layer 2   h1 (all 256 columns, from LDS) x the wave's W2 slice, + b2,
//             ReLU, bf16 -> the wave's h2 columns in LDS
//   head      the wave's 32 h2 columns x W3 rows 32w.. (one k block): a
//             partial [64 x 4], summed over the 8 waves in wave order (so
//             scores do not depend on timing), softmax, score
// Two workgroup barriers per tile.  Rounding points as everywhere else: h1
// and h2 in bf16, fp32 sums.
// ---------------------------------------------------------------------------
constexpr int kSc2Waves = 8;
constexpr int kSc2Rows = 64;
constexpr int kSc2Pitch = kMlpHidden + 8;   // bf16 per LDS row (16-lane reads conflict-free)

// LDS writes of the wave before this point are seen by its reads after it
// (a wave's LDS operations complete in order; only the compiler is held).
__device__ __forceinline__ void mlp_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bf16x8 load_bf16x8(const uint16_t* p)
{
    return *reinterpret_cast<const bf16x8*>(p);
}

// One-hot A operand of k block kb for a genome: lane group q = l / 16 holds
// edge e = 4 kb + q, so its 8 values are 1.0 at that edge's colour (none if
// the edge is absent).
__device__ __forceinline__ bf16x8 onehot_operand(uint64_t g, int t, int bits, uint32_t cmask,
                                                 int e)
{
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if (e < 4 * t) {
        const uint32_t colour = (uint32_t)(g >> (bits * (4 * t - 1 - e))) & cmask;
        // colour < 8 for every c the network takes (its input has 8 slots per edge)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            w[q] = (colour == 2u * q ? 0x3F80u : 0u) | (colour == 2u * q + 1u ? 0x3F800000u : 0u);
    }
    bf16x8 v;
    __builtin_memcpy(&v, w, sizeof(v));
    return v;
}

// kind: JATAM_PREDICT_SCREEN, _COST or _P_UNBOUND (what is written per genome).
template <int KB1>
__global__ __launch_bounds__(512) void mlp_score_persistent_kernel(MlpArgs a,
                                                                   const uint64_t* genomes,
                                                                   const uint8_t* tvec, int t_all,
                                                                   uint32_t n, float* scores,
                                                                   int kind)
{
    __shared__ __attribute__((aligned(16))) uint16_t h1s[kSc2Rows][kSc2Pitch];
    __shared__ __attribute__((aligned(16))) uint16_t h2s[kSc2Rows][kSc2Pitch];
    __shared__ float part[kSc2Waves][kSc2Rows][kMlpOut];
    const int tid = (int)threadIdx.x, wave = tid >> 6, l = tid & 63;
    const int r16 = l & 15, q = l >> 4;
    const int col0 = 32 * wave;
    const uint32_t cmask = (uint32_t)a.c - 1u;
    // the wave's weights, as B operands: lane holds B[8q + i][r16] of each block
    bf16x8 w1f[KB1][2], w2f[8][2], w3f;
#pragma unroll
    for (int kb = 0; kb < KB1; ++kb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            uint16_t v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                v[i] = a.w1b[(size_t)(32 * kb + 8 * q + i) * kMlpHidden + col0 + 16 * nb + r16];
            __builtin_memcpy(&w1f[kb][nb], v, sizeof(v));
        }
#pragma unroll
    for (int kb = 0; kb < 8; ++kb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
            w2f[kb][nb] = load_bf16x8(a.w2t + (size_t)(col0 + 16 * nb + r16) * kMlpHidden +
                                      32 * kb + 8 * q);
    w3f = load_bf16x8(a.w3t + (size_t)r16 * kMlpHidden + col0 + 8 * q);
    const float b1v[2] = {a.p.b1[col0 + r16], a.p.b1[col0 + 16 + r16]};
    const float b2v[2] = {a.p.b2[col0 + r16], a.p.b2[col0 + 16 + r16]};
    const float b3v = tid < kSc2Rows * kMlpOut ? a.p.b3[tid & 3] : 0.f;

    const uint32_t tiles = (n + kSc2Rows - 1) / kSc2Rows;
    for (uint32_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const uint32_t s0 = tile * kSc2Rows;
        // -- layer 1: one-hot x W1 ----------------------------------------
        floatx4 acc[4][2];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const uint32_t sidx = s0 + (uint32_t)(16 * mb + r16);
            uint64_t g = 0;
            int t = 0;
            if (sidx < n) {
                g = genomes[sidx];
                t = mlp_tiles(tvec != nullptr ? tvec[sidx] : t_all);
            }
            acc[mb][0] = floatx4{0.f, 0.f, 0.f, 0.f};
            acc[mb][1] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < KB1; ++kb) {
                const bf16x8 x = onehot_operand(g, t, a.bits, cmask, 4 * kb + q);
                acc[mb][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, w1f[kb][0], acc[mb][0],
                                                                     0, 0, 0);
                acc[mb][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, w1f[kb][1], acc[mb][1],
                                                                     0, 0, 0);
            }
        }
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float z = acc[mb][nb][i] + b1v[nb];
                    h1s[16 * mb + 4 * q + i][col0 + 16 * nb + r16] = bf16_bits(z > 0.f ? z : 0.f);
                }
        __syncthreads();   // h1 complete; the previous tile's partial heads consumed
        // -- layer 2: h1 x W2 (the wave's columns) ------------------------
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            acc[mb][0] = floatx4{0.f, 0.f, 0.f, 0.f};
            acc[mb][1] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                const bf16x8 af = load_bf16x8(&h1s[16 * mb + r16][32 * kb + 8 * q]);
                acc[mb][0] =
                    __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, w2f[kb][0], acc[mb][0], 0, 0, 0);
                acc[mb][1] =
                    __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, w2f[kb][1], acc[mb][1], 0, 0, 0);
            }
        }
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float z = acc[mb][nb][i] + b2v[nb];
                    h2s[16 * mb + 4 * q + i][col0 + 16 * nb + r16] = bf16_bits(z > 0.f ? z : 0.f);
                }
        mlp_wave_sync();   // the wave reads back only its own h2 columns
        // -- head: the wave's partial h2 W3 -------------------------------
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const bf16x8 af = load_bf16x8(&h2s[16 * mb + r16][col0 + 8 * q]);
            const floatx4 o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                af, w3f, floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            if (r16 < kMlpOut)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    part[wave][16 * mb + 4 * q + i][r16] = o[i];
        }
        __syncthreads();   // partial heads complete; h1 free for the next tile
        if (tid < kSc2Rows * kMlpOut) {
            const int row = tid >> 2, o = tid & 3;
            float v = 0.f;
#pragma unroll
            for (int w = 0; w < kSc2Waves; ++w)
                v += part[w][row][o];
            v += b3v;
            // gather the row's four outputs in its lane quad
            const float o0 = __shfl(v, (l & ~3) + 0), o1 = __shfl(v, (l & ~3) + 1);
            const float o2 = __shfl(v, (l & ~3) + 2), o3 = __shfl(v, (l & ~3) + 3);
            if (o == 0 && s0 + (uint32_t)row < n) {
                const float mx = fmaxf(o0, fmaxf(o1, o2));
                const float e0 = expf(o0 - mx), e1 = expf(o1 - mx), e2 = expf(o2 - mx);
                const float inv = 1.f / (e0 + e1 + e2);
                scores[s0 + row] = kind == JATAM_PREDICT_COST        ? expf(o3) - 1.f
                                   : kind == JATAM_PREDICT_P_UNBOUND ? e0 * inv
                                                                     : e2 * inv * expf(o3) - 1.f;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Head and loss: out = h2 W3 + b3 per sample; with labels, the per-sample loss
// and dout = d(mean loss)/d(out).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mlp_head_kernel(MlpArgs a, uint32_t n,
                                                       const jatam_result_t* labels,
                                                       float* out4, float* scores)
{
    const uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= n)
        return;
    float o[kMlpOut];
#pragma unroll
    for (int k = 0; k < kMlpOut; ++k)
        o[k] = a.p.b3[k];
    const uint16_t* h = a.h2 + (size_t)b * kMlpHidden;
    for (int j = 0; j < kMlpHidden; ++j) {
        const float hj = bf16_float(h[j]);
#pragma unroll
        for (int k = 0; k < kMlpOut; ++k)
            o[k] = fmaf(hj, bf16_float(a.w3b[j * kMlpOut + k]), o[k]);
    }
    if (out4 != nullptr)
#pragma unroll
        for (int k = 0; k < kMlpOut; ++k)
            out4[(size_t)b * kMlpOut + k] = o[k];
    if (scores != nullptr) {
        // expected size of a deterministic structure: P(DET) e^pred - 1
        const float mx = fmaxf(o[0], fmaxf(o[1], o[2]));
        const float e0 = expf(o[0] - mx), e1 = expf(o[1] - mx), e2 = expf(o[2] - mx);
        scores[b] = e2 / (e0 + e1 + e2) * expf(o[3]) - 1.f;
    }
    if (labels == nullptr)
        return;
    const jatam_result_t rec = labels[b];
    const int y = rec.cls == JATAM_UNBOUND ? 0 : rec.cls == JATAM_DET ? 2 : 1;
    const float mx = fmaxf(o[0], fmaxf(o[1], o[2]));
    const float e0 = expf(o[0] - mx), e1 = expf(o[1] - mx), e2 = expf(o[2] - mx);
    const float s = e0 + e1 + e2;
    const float py = (y == 0 ? e0 : y == 1 ? e1 : e2) / s;
    const float target = log1pf((float)rec.size);
    const float err = o[3] - target;
    a.loss[b] = -logf(py) + err * err;
    const float inv = 1.f / (float)n;
    a.dout[(size_t)b * kMlpOut + 0] = (e0 / s - (y == 0 ? 1.f : 0.f)) * inv;
    a.dout[(size_t)b * kMlpOut + 1] = (e1 / s - (y == 1 ? 1.f : 0.f)) * inv;
    a.dout[(size_t)b * kMlpOut + 2] = (e2 / s - (y == 2 ? 1.f : 0.f)) * inv;
    a.dout[(size_t)b * kMlpOut + 3] = 2.f * err * inv;
}

// dh2 = bf16((dout W3^T) * (h2 > 0)), one thread per (sample, unit); zero on
// padding rows (b >= n).
__global__ __launch_bounds__(256) void mlp_dh2_kernel(MlpArgs a, uint32_t n)
{
    const uint32_t b = blockIdx.x;
    const int j = threadIdx.x;
    if (b >= n) {
        a.dh2[(size_t)b * kMlpHidden + j] = 0;
        return;
    }
    float v = 0.f;
#pragma unroll
    for (int k = 0; k < kMlpOut; ++k)
        v = fmaf(a.dout[(size_t)b * kMlpOut + k], bf16_float(a.w3b[j * kMlpOut + k]), v);
    const size_t o = (size_t)b * kMlpHidden + j;
    a.dh2[o] = bf16_bits(a.h2[o] != 0 ? v : 0.f);
}

// Row chunks of the batch reductions below: each block sums one chunk of
// rows into partial[chunk][...]; mlp_reduce_kernel adds the chunks in order.
constexpr int kRedRows = 128;

// Column sums of [n][cols] rows (bf16 or fp32): partial[chunk][j].
__global__ __launch_bounds__(256) void mlp_colsum_kernel(const uint16_t* src16, const float* src32,
                                                         uint32_t n, int cols, float* partial)
{
    const uint32_t b0 = blockIdx.y * kRedRows, b1 = min(n, b0 + kRedRows);
    for (int j = blockIdx.x * 256 + threadIdx.x; j < cols; j += gridDim.x * 256) {
        float s = 0.f;
        for (uint32_t b = b0; b < b1; ++b)
            s += src16 != nullptr ? bf16_float(src16[(size_t)b * cols + j])
                                  : src32[(size_t)b * cols + j];
        partial[(size_t)blockIdx.y * cols + j] = s;
    }
}

// dW3[j][k] = sum_b h2[b][j] dout[b][k]: partial[chunk][j * 4 + k].
__global__ __launch_bounds__(256) void mlp_dw3_kernel(MlpArgs a, uint32_t n, float* partial)
{
    const int j = threadIdx.x;
    const uint32_t b0 = blockIdx.x * kRedRows, b1 = min(n, b0 + kRedRows);
    float s[kMlpOut] = {0.f, 0.f, 0.f, 0.f};
    for (uint32_t b = b0; b < b1; ++b) {
        const float h = bf16_float(a.h2[(size_t)b * kMlpHidden + j]);
#pragma unroll
        for (int k = 0; k < kMlpOut; ++k)
            s[k] = fmaf(h, a.dout[(size_t)b * kMlpOut + k], s[k]);
    }
#pragma unroll
    for (int k = 0; k < kMlpOut; ++k)
        partial[(size_t)blockIdx.x * kMlpHidden * kMlpOut + j * kMlpOut + k] = s[k];
}

// Per-chunk loss sums: partial[chunk].
__global__ __launch_bounds__(256) void mlp_loss_kernel(MlpArgs a, uint32_t n, float* partial)
{
    __shared__ float part[256];
    const uint32_t b0 = blockIdx.x * kRedRows, b1 = min(n, b0 + kRedRows);
    const uint32_t b = b0 + threadIdx.x;
    part[threadIdx.x] = b < b1 ? a.loss[b] : 0.f;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        partial[blockIdx.x] = part[0];
}

// loss_out = (sum of the chunk sums) / n.
__global__ void mlp_loss_final_kernel(const float* partial, int chunks, uint32_t n,
                                      float* loss_out)
{
    if (threadIdx.x != 0)
        return;
    float s = 0.f;
    for (int c = 0; c < chunks; ++c)
        s += partial[c];
    loss_out[0] = s / (float)n;
}

// Adam on the flat fp32 parameter vector; refreshes the bf16 weight copies.
__global__ __launch_bounds__(256) void mlp_adam_kernel(MlpArgs a, float lr, float bc1, float bc2)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kMlpParams)
        return;
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    const float gi = a.g.flat[i];
    const float m = beta1 * a.m[i] + (1.f - beta1) * gi;
    const float v = beta2 * a.v[i] + (1.f - beta2) * gi * gi;
    a.m[i] = m;
    a.v[i] = v;
    const float w = a.p.flat[i] - lr * (m / bc1) / (sqrtf(v / bc2) + eps);
    a.p.flat[i] = w;
    refresh_bf16(a, i, w);
}

// bf16 copies of all weights from the fp32 masters.
__global__ __launch_bounds__(256) void mlp_refresh_kernel(MlpArgs a)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < kMlpParams)
        refresh_bf16(a, i, a.p.flat[i]);
}

// The library's own initialisation: He-uniform weights from Philox words,
// w = (2u - 1) sqrt(6 / fan_in) with u = word / 2^32; biases zero.
__global__ __launch_bounds__(256) void mlp_init_kernel(MlpArgs a, uint32_t k0, uint32_t k1)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kMlpParams)
        return;
    float w = 0.f;
    int fan_in = 0;
    if (i < kMlpOffB1)
        fan_in = kMlpIn;
    else if (i >= kMlpOffW2 && i < kMlpOffB2)
        fan_in = kMlpHidden;
    else if (i >= kMlpOffW3 && i < kMlpOffB3)
        fan_in = kMlpHidden;
    if (fan_in) {
        const Words4 r = philox4x32_10((uint32_t)i, 0, 0, 3u << 28, k0, k1);
        const float u = (float)(r.w[0] >> 8) * (1.f / 16777216.f);
        w = (2.f * u - 1.f) * sqrtf(6.f / (float)fan_in);
    }
    a.p.flat[i] = w;
    a.m[i] = 0.f;
    a.v[i] = 0.f;
    refresh_bf16(a, i, w);
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
// C = A B (M x N, K a multiple of 32, M and N multiples of 8).  Store
// epilogues with a long K are split across workgroups (fp32 partials in
// `partial`, added in split order).
static int gemm(GemmArgs g, float* partial, hipStream_t s)
{
    const int tiles = ((g.M + kBM - 1) / kBM) * ((g.N + kBN - 1) / kBN);
    g.splits = 1;
    if (g.epilogue == kEpStoreF32) {
        const int want = g.K / 256;
        g.splits = want < 1 ? 1 : want > 16 ? 16 : want;
    }
    g.partial = partial;
    hipLaunchKernelGGL(mlp_gemm_kernel, dim3(tiles, g.splits), dim3(256), 0, s, g);
    if (g.splits > 1) {
        const int64_t count = (int64_t)g.M * g.N;
        hipLaunchKernelGGL(mlp_reduce_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                           s, (const float*)partial, g.splits, count, g.C32);
    }
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

size_t mlp_partial_floats(size_t max_batch)
{
    const size_t chunks = (max_batch + kRedRows - 1) / kRedRows;
    const size_t split = (size_t)16 * kMlpHidden * kMlpHidden;       // dW2, 16 splits
    const size_t rows = chunks * (size_t)(kMlpHidden * kMlpOut);      // dW3 chunk sums
    return split > rows ? split : rows;
}

// Sum of `chunks` partial rows of `cols` floats into out (fixed order).
static void reduce_rows(const float* partial, int chunks, int cols, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, s,
                       partial, chunks, (int64_t)cols, out);
}

int mlp_launch_init(const MlpArgs& a, uint64_t seed, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_init_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, a,
                       (uint32_t)seed, (uint32_t)(seed >> 32));
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

int mlp_launch_refresh(const MlpArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_refresh_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

// Forward pass over n samples (n a multiple of 16); out4 may be null.
// Forward pass over n samples padded to n_pad (a multiple of 32): padding rows
// carry zero inputs and are never read back; out4 may be null.
int mlp_launch_forward(const MlpArgs& a, const uint64_t* genomes, const uint8_t* tvec, int t_all,
                       uint32_t n, uint32_t n_pad, const jatam_result_t* labels, float* out4,
                       hipStream_t s)
{
    hipLaunchKernelGGL(mlp_layer1_kernel, dim3(n_pad), dim3(256), 0, s, a, genomes, tvec, t_all,
                       n);
    GemmArgs g{};
    g.A = a.h1;
    g.sam = kMlpHidden;
    g.sak = 1;
    g.B = a.w2b;
    g.sbk = kMlpHidden;
    g.sbn = 1;
    g.M = (int)n_pad;
    g.N = kMlpHidden;
    g.K = kMlpHidden;
    g.epilogue = kEpBiasRelu;
    g.C16 = a.h2;
    g.bias = a.p.b2;
    int rc = gemm(g, a.partial, s);
    if (rc != JATAM_OK)
        return rc;
    hipLaunchKernelGGL(mlp_head_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a, n, labels,
                       out4, (float*)nullptr);
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

// Predictions of n samples (any n; no padding, no activations kept).
int mlp_launch_score(const MlpArgs& a, const uint64_t* genomes, const uint8_t* tvec, int t_all,
                     uint32_t n, float* scores, int kind, hipStream_t s)
{
    if (n == 0)
        return JATAM_OK;
    // k blocks of the one-hot input that can be nonzero: 4 edges per block
    const int kb1 = tvec != nullptr ? 3 : t_all;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return JATAM_E_HIP;
    const void* fn = kb1 == 1   ? (const void*)mlp_score_persistent_kernel<1>
                     : kb1 == 2 ? (const void*)mlp_score_persistent_kernel<2>
                                : (const void*)mlp_score_persistent_kernel<3>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 512, 0) != hipSuccess)
        return JATAM_E_HIP;
    per_cu = per_cu < 1 ? 1 : per_cu;
    const uint32_t tiles = (n + kSc2Rows - 1) / kSc2Rows;
    const uint32_t blocks = tiles < (uint32_t)(cus * per_cu) ? tiles : (uint32_t)(cus * per_cu);
    if (kb1 == 1)
        hipLaunchKernelGGL(mlp_score_persistent_kernel<1>, dim3(blocks), dim3(512), 0, s, a,
                           genomes, tvec, t_all, n, scores, kind);
    else if (kb1 == 2)
        hipLaunchKernelGGL(mlp_score_persistent_kernel<2>, dim3(blocks), dim3(512), 0, s, a,
                           genomes, tvec, t_all, n, scores, kind);
    else
        hipLaunchKernelGGL(mlp_score_persistent_kernel<3>, dim3(blocks), dim3(512), 0, s, a,
                           genomes, tvec, t_all, n, scores, kind);
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

// Backward pass of the last forward (with labels).
int mlp_launch_backward(const MlpArgs& a, uint32_t n, uint32_t n_pad, float* loss_out,
                        hipStream_t s)
{
    const int chunks = (int)((n + kRedRows - 1) / kRedRows);
    const int chunks_pad = (int)((n_pad + kRedRows - 1) / kRedRows);
    if (loss_out != nullptr) {
        hipLaunchKernelGGL(mlp_loss_kernel, dim3(chunks), dim3(256), 0, s, a, n, a.partial);
        hipLaunchKernelGGL(mlp_loss_final_kernel, dim3(1), dim3(64), 0, s, (const float*)a.partial,
                           chunks, n, loss_out);
    }
    hipLaunchKernelGGL(mlp_dw3_kernel, dim3(chunks), dim3(kMlpHidden), 0, s, a, n, a.partial);
    reduce_rows(a.partial, chunks, kMlpHidden * kMlpOut, a.g.w3, s);
    hipLaunchKernelGGL(mlp_colsum_kernel, dim3(1, chunks), dim3(256), 0, s,
                       (const uint16_t*)nullptr, (const float*)a.dout, n, kMlpOut, a.partial);
    reduce_rows(a.partial, chunks, kMlpOut, a.g.b3, s);
    hipLaunchKernelGGL(mlp_dh2_kernel, dim3(n_pad), dim3(256), 0, s, a, n);
    // dW2 = h1^T dh2 (M = K_hidden rows of h1^T, K = batch)
    GemmArgs g{};
    g.A = a.h1;
    g.sam = 1;
    g.sak = kMlpHidden;
    g.B = a.dh2;
    g.sbk = kMlpHidden;
    g.sbn = 1;
    g.M = kMlpHidden;
    g.N = kMlpHidden;
    g.K = (int)n_pad;
    g.epilogue = kEpStoreF32;
    g.C32 = a.g.w2;
    int rc = gemm(g, a.partial, s);
    if (rc != JATAM_OK)
        return rc;
    hipLaunchKernelGGL(mlp_colsum_kernel, dim3(1, chunks_pad), dim3(256), 0, s,
                       (const uint16_t*)a.dh2, (const float*)nullptr, n_pad, kMlpHidden,
                       a.partial);
    reduce_rows(a.partial, chunks_pad, kMlpHidden, a.g.b2, s);
    // dh1 = bf16((dh2 W2^T) * (h1 > 0))
    g = GemmArgs{};
    g.A = a.dh2;
    g.sam = kMlpHidden;
    g.sak = 1;
    g.B = a.w2b;
    g.sbk = 1;
    g.sbn = kMlpHidden;
    g.M = (int)n_pad;
    g.N = kMlpHidden;
    g.K = kMlpHidden;
    g.epilogue = kEpReluMask;
    g.C16 = a.dh1;
    g.mask = a.h1;
    if ((rc = gemm(g, a.partial, s)) != JATAM_OK)
        return rc;
    hipLaunchKernelGGL(mlp_colsum_kernel, dim3(1, chunks_pad), dim3(256), 0, s,
                       (const uint16_t*)a.dh1, (const float*)nullptr, n_pad, kMlpHidden,
                       a.partial);
    reduce_rows(a.partial, chunks_pad, kMlpHidden, a.g.b1, s);
    // dW1 = x^T dh1
    g = GemmArgs{};
    g.A = a.x;
    g.sam = 1;
    g.sak = kMlpIn;
    g.B = a.dh1;
    g.sbk = kMlpHidden;
    g.sbn = 1;
    g.M = kMlpIn;
    g.N = kMlpHidden;
    g.K = (int)n_pad;
    g.epilogue = kEpStoreF32;
    g.C32 = a.g.w1;
    return gemm(g, a.partial, s);
}

int mlp_launch_adam(const MlpArgs& a, float lr, int step, hipStream_t s)
{
    const float bc1 = 1.f - powf(0.9f, (float)step);
    const float bc2 = 1.f - powf(0.999f, (float)step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, a, lr,
                       bc1, bc2);
    return hipGetLastError() == hipSuccess ? JATAM_OK : JATAM_E_HIP;
}

}  // namespace jatam
