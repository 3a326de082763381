// Pair-scoring MLP on MFMA: x = [sig_a XOR sig_b, sig_a AND sig_b] (8,192
// bits) -> 512 -> 256 -> 1, ReLU, BF16 weights and activations as matrix
// operands, FP32 accumulation, FP32 master weights updated by Adam.
//
// Every matrix product is written in "NT" form, C[m][n] = sum_k A(m,k)B(n,k),
// with both operands contiguous along k, so each lane of a
// v_mfma_f32_32x32x16_bf16 tile reads its eight k-consecutive values with
// one 16-byte load (or expands them from eight signature bits).  Layouts:
//   W1 [512][8192], W2 [256][512] (out x in) for the forward products,
//   W2T [512][256] for the input gradient of layer 2,
//   activations stored row-major and, where a weight gradient needs them as
//   the k-contiguous operand, also transposed.
// Reductions over the batch (bias and head gradients) run in a fixed order,
// so training is deterministic.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mlp_kernels.h"

namespace kripke {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
  // round to nearest even (inputs are finite)
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 as_bf16x8(u16x8 v) { return __builtin_bit_cast(bf16x8, v); }

// 8 bits -> eight bf16 values 1.0 / 0.0
__device__ __forceinline__ bf16x8 expand_bits(uint32_t byte) {
  u16x8 v;
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = ((byte >> j) & 1u) ? 0x3F80u : 0u;
  return as_bf16x8(v);
}

// ------------------------------------------------------------ loaders
struct Dense {  // row-major [rows][ld] bf16, k-contiguous
  const uint16_t* p;
  uint32_t ld, rows;
  __device__ __forceinline__ bf16x8 load(uint32_t row, uint32_t k0) const {
    if (row >= rows) return as_bf16x8(u16x8(0));
    return as_bf16x8(*reinterpret_cast<const u16x8*>(p + (uint64_t)row * ld + k0));
  }
};

// Row m of the pair input: bit k of x_m (k < 4096: XOR, else AND).
struct PairRows {
  const uint64_t* sig;
  const uint64_t* pairs;
  uint32_t rows;
  __device__ __forceinline__ bf16x8 load(uint32_t row, uint32_t k0) const {
    if (row >= rows) return as_bf16x8(u16x8(0));
    const uint64_t pr = pairs[row];
    const uint64_t* a = sig + (pr >> 32) * kSigWords;
    const uint64_t* b = sig + (pr & 0xFFFFFFFFu) * kSigWords;
    const uint32_t k = k0 & 4095u, w = k >> 6, sh = k & 63u;
    const uint64_t x = k0 < 4096 ? (a[w] ^ b[w]) : (a[w] & b[w]);
    return expand_bits((uint32_t)(x >> sh) & 0xFFu);
  }
};

// Row f of the transposed pair input: bit f of x_m for m = k0 .. k0+7.
struct PairCols {
  const uint64_t* sig;
  const uint64_t* pairs;
  uint32_t npairs;
  __device__ __forceinline__ bf16x8 load(uint32_t f, uint32_t k0) const {
    if (f >= kIn) return as_bf16x8(u16x8(0));
    const uint32_t k = f & 4095u, w = k >> 6, sh = k & 63u;
    uint32_t byte = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t m = k0 + j;
      if (m >= npairs) continue;
      const uint64_t pr = pairs[m];
      const uint64_t a = sig[(pr >> 32) * kSigWords + w], b = sig[(pr & 0xFFFFFFFFu) * kSigWords + w];
      const uint64_t x = f < 4096 ? (a ^ b) : (a & b);
      byte |= (uint32_t)((x >> sh) & 1u) << j;
    }
    return expand_bits(byte);
  }
};

// ----------------------------------------------------------- epilogues
// Layer output: a = relu(acc + bias); bf16 row-major, optional bf16
// transposed and fp32 row-major copies.
struct EpiHidden {
  const float* bias;
  uint16_t* out;     // [M][N]
  uint16_t* out_t;   // [N][ldt] or null
  float* out_f;      // [M][N] or null
  uint32_t N, ldt;
  __device__ __forceinline__ void store(uint32_t m, uint32_t n, float acc) const {
    const float a = fmaxf(acc + bias[n], 0.0f);
    const uint16_t h = to_bf16(a);
    out[(uint64_t)m * N + n] = h;
    if (out_t) out_t[(uint64_t)n * ldt + m] = h;
    if (out_f) out_f[(uint64_t)m * N + n] = a;
  }
};

// Input gradient of a ReLU layer: d = acc where the stored activation is
// positive, else 0; fp32 row-major (for the bias gradient) and bf16
// transposed (operand of the weight gradient).
struct EpiReluGrad {
  const uint16_t* act;  // [M][N] bf16 activations of that layer
  float* out_f;         // [M][N]
  uint16_t* out_t;      // [N][ldt]
  uint32_t N, ldt;
  __device__ __forceinline__ void store(uint32_t m, uint32_t n, float acc) const {
    const float d = from_bf16(act[(uint64_t)m * N + n]) > 0.0f ? acc : 0.0f;
    out_f[(uint64_t)m * N + n] = d;
    out_t[(uint64_t)n * ldt + m] = to_bf16(d);
  }
};

struct EpiStore {  // plain fp32 row-major
  float* out;
  uint32_t N;
  __device__ __forceinline__ void store(uint32_t m, uint32_t n, float acc) const {
    out[(uint64_t)m * N + n] = acc;
  }
};

// ---------------------------------------------------------------- GEMM
// Block = 4 waves = a 128x128 tile of C; each wave a 64x64 tile, i.e. 2x2
// MFMA tiles of 32x32, so every operand fragment it loads (or expands from
// signature bits) feeds two MFMAs.  Lane l supplies A(row = l % 32,
// k = k0 + 8 (l / 32) .. +7) for each of its two row tiles and likewise B;
// accumulator register r of lane l is C(8 (r / 4) + 4 (l / 32) + r % 4, l % 32)
// of its tile.  Every element accumulates the same MFMA sequence over k as
// with one tile per wave, so results do not depend on the tiling.
template <class LA, class LB, class EPI, int TM, int TN>
__global__ __launch_bounds__(256) void gemm_nt(LA A, LB B, EPI E, uint32_t M, uint32_t N,
                                                uint32_t K) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t m0 = blockIdx.x * (64 * TM) + (wv & 1) * (32 * TM);
  const uint32_t n0 = blockIdx.y * (64 * TN) + (wv >> 1) * (32 * TN);
  const uint32_t kh = 8 * (lane >> 5);
  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x16{0};
  for (uint32_t k0 = 0; k0 < K; k0 += 16) {
    bf16x8 a[TM], b[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) a[i] = A.load(m0 + 32 * i + (lane & 31), k0 + kh);
#pragma unroll
    for (int j = 0; j < TN; ++j) b[j] = B.load(n0 + 32 * j + (lane & 31), k0 + kh);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint32_t m = m0 + 32 * i + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
        const uint32_t n = n0 + 32 * j + (lane & 31);
        if (m < M && n < N) E.store(m, n, acc[i][j][r]);
      }
}

// TM x TN MFMA tiles per wave (block tile 64 TM x 64 TN)
template <int TM, int TN, class LA, class LB, class EPI>
hipError_t gemm_tiles(LA A, LB B, EPI E, uint32_t M, uint32_t N, uint32_t K, hipStream_t s) {
  dim3 grid((M + 64 * TM - 1) / (64 * TM), (N + 64 * TN - 1) / (64 * TN));
  hipLaunchKernelGGL((gemm_nt<LA, LB, EPI, TM, TN>), grid, dim3(256), 0, s, A, B, E, M, N, K);
  return hipGetLastError();
}

// Larger per-wave tiles reuse each operand fragment for more MFMAs but make
// fewer blocks: they are used only while the grid still has at least four
// blocks per CU (training batches of a few hundred pairs keep one tile per
// wave).  Every element accumulates the same MFMA sequence either way.
template <int TM = 2, int TN = 2, class LA, class LB, class EPI>
hipError_t gemm(LA A, LB B, EPI E, uint32_t M, uint32_t N, uint32_t K, hipStream_t s) {
  if (M == 0 || N == 0) return hipSuccess;
  auto blocks = [&](uint32_t tm, uint32_t tn) {
    return (uint64_t)((M + 64 * tm - 1) / (64 * tm)) * ((N + 64 * tn - 1) / (64 * tn));
  };
  if (blocks(TM, TN) >= 1024) return gemm_tiles<TM, TN>(A, B, E, M, N, K, s);
  if (blocks(2, 2) >= 1024) return gemm_tiles<2, 2>(A, B, E, M, N, K, s);
  return gemm_tiles<1, 1>(A, B, E, M, N, K, s);
}

// ------------------------------------------- scoring: layer 2 and head
// Scoring forward of layers 2 and 3 without storing layer 2's activations:
// each MFMA tile covers 32 outputs of 32 rows, and the lanes l with the same
// l / 32 hold the same rows (lane l % 32 one output each), so a butterfly over
// l % 32 reduces relu(acc + b2) * w3 of a row over the tile's 32 outputs in a
// fixed order; lane 0 of each half-wave writes that partial for its rows:
// part[m][g] = sum over outputs n = 32 g .. 32 g + 31.  The tile of an output
// group is the same whatever tiles per wave the grid uses, so the partials,
// and head_sum's logits, do not depend on the tiling.
constexpr int kHeadGroups = kH2 / 32;  // 32-output groups of layer 2

template <int TM, int TN>
__global__ __launch_bounds__(256) void gemm_l2_head(Dense A, Dense B, const float* b2,
                                                     const float* w3, float* part, uint32_t M) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // XCD-aware order: the column blocks of one row block run back to back on
  // the same XCD (blocks are dealt to the 8 XCDs round-robin), so the row
  // block's activations come from HBM once and from that XCD's L2 after
  constexpr uint32_t CB = kH2 / (64 * TN);
  const uint32_t xcd = blockIdx.x & 7u, q = blockIdx.x >> 3;
  const uint32_t rb = (q / CB) * 8 + xcd, cb = q % CB;
  const uint32_t m0 = rb * (64 * TM) + (wv & 1) * (32 * TM);
  const uint32_t n0 = cb * (64 * TN) + (wv >> 1) * (32 * TN);
  const uint32_t kh = 8 * (lane >> 5);
  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x16{0};
  // steps of 64 k (four MFMA k-slices); the next step's fragments are loaded
  // into registers while this step's MFMAs run
  constexpr uint32_t kStep = 64;
  bf16x8 xa[4][TM], xb[4][TN], ya[4][TM], yb[4][TN];
  auto fetch = [&](bf16x8 (&fa)[4][TM], bf16x8 (&fb)[4][TN], uint32_t k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int i = 0; i < TM; ++i) fa[q][i] = A.load(m0 + 32 * i + (lane & 31), k0 + 16 * q + kh);
#pragma unroll
      for (int j = 0; j < TN; ++j) fb[q][j] = B.load(n0 + 32 * j + (lane & 31), k0 + 16 * q + kh);
    }
  };
  fetch(xa, xb, 0);
  for (uint32_t k0 = 0; k0 < kH1; k0 += kStep) {
    const bool more = k0 + kStep < kH1;
    if (more) fetch(ya, yb, k0 + kStep);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[q][i], xb[q][j], acc[i][j], 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
    if (more) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int i = 0; i < TM; ++i) xa[q][i] = ya[q][i];
#pragma unroll
        for (int j = 0; j < TN; ++j) xb[q][j] = yb[q][j];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const uint32_t n = n0 + 32 * j + (lane & 31);
    const float bn = b2[n], wn = w3[n];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        float v = fmaxf(acc[i][j][r] + bn, 0.0f) * wn;
#pragma unroll
        for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o);
        const uint32_t m = m0 + 32 * i + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
        if ((lane & 31) == 0 && m < M) part[(uint64_t)m * kHeadGroups + (n0 + 32 * j) / 32] = v;
      }
  }
}

// logit[m] = b3 + the row's output-group partials, summed in group order.
__global__ void head_sum(const float* part, const float* b3, uint32_t M, float* logit) {
  const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  float s = 0.0f;
#pragma unroll
  for (int g = 0; g < kHeadGroups; ++g) s += part[(uint64_t)m * kHeadGroups + g];
  logit[m] = s + b3[0];
}

template <int TM, int TN>
hipError_t l2_head_tiles(Dense A, Dense B, const float* b2, const float* w3, float* part,
                         uint32_t M, hipStream_t s) {
  // row blocks padded to a multiple of 8 (the padding blocks' rows are past M:
  // zero operands, nothing stored)
  const uint32_t rbs = ((M + 64 * TM - 1) / (64 * TM) + 7) / 8 * 8;
  const uint32_t grid = rbs * (kH2 / (64 * TN));
  hipLaunchKernelGGL((gemm_l2_head<TM, TN>), dim3(grid), dim3(256), 0, s, A, B, b2, w3, part, M);
  return hipGetLastError();
}

// The same tile choice as gemm(): 2 x 2 tiles per wave while the grid keeps
// at least 1,024 blocks, else one.
hipError_t l2_head(Dense A, Dense B, const float* b2, const float* w3, float* part, uint32_t M,
                   hipStream_t s) {
  if (M == 0) return hipSuccess;
  const uint64_t wide = (uint64_t)((M + 127) / 128) * (kH2 / 128);
  return wide >= 1024 ? l2_head_tiles<2, 2>(A, B, b2, w3, part, M, s)
                      : l2_head_tiles<1, 1>(A, B, b2, w3, part, M, s);
}

// ------------------------------------------------------ layer-1 forward
// C[m][n] = sum_k x_m(k) W1[n][k] for the scoring and training forwards of
// large batches: M pairs x 512 outputs x K = 8,192, where x_m(k) is bit k of
// [sig_a XOR sig_b, sig_a AND sig_b].  W1 is the only operand worth staging:
// a block covers 256 pairs x 128 outputs and stages W1[n0 .. n0+127][k0 ..
// k0+63] in LDS per step, double-buffered (the next step's tile is loaded
// into registers while this step's MFMAs run), so each W1 byte fetched from
// L2 feeds 256 pairs.  Each of the 4 waves owns 64 pairs x 128 outputs (2 x 4
// MFMA tiles of 32 x 32); its pair operands come from one 64-bit signature
// word per pair and step (fetched a step ahead), expanded 8 bits at a time to
// BF16 0/1 fragments.  Rows are padded to 144 bytes so the 16-byte fragment
// reads of 16 consecutive rows hit 16 distinct 4-bank groups.
// Block order is XCD-aware: the 8 XCDs take blocks round-robin, and XCDs x
// and x + 4 both work on output quarter x & 3, so each XCD's L2 holds a
// quarter of W1 (2 MB) instead of all of it.
// Every output accumulates the same v_mfma_f32_32x32x16_bf16 sequence over k
// (ascending steps of 16, same fragment layout) as gemm_nt, so the result is
// bitwise the same as with gemm_nt.
constexpr int kW1BM = 256, kW1BN = 128, kW1BK = 64, kW1Pad = kW1BK + 8;

__device__ __forceinline__ bf16x8 expand_byte(uint32_t byte) {
  // bits 2j, 2j+1 -> dword j = {bf16(bit 2j), bf16(bit 2j+1)}.  t = byte +
  // (byte << 15) holds bit 2j at 2j and bit 2j+1 at 16 + 2j; masking those
  // two and one 24-bit multiply by 0x3F80 >> 2j (1.0 in BF16, whose low
  // seven bits are zero, so the shift is exact) moves them to bits 0 and 16
  // as BF16 values: two instructions per dword.
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  const uint32_t t = __umul24(byte, 0x8001u);
  u32x4 d;
#pragma unroll
  for (int j = 0; j < 4; ++j) d[j] = __umul24(t & (0x10001u << (2 * j)), 0x3F80u >> (2 * j));
  return __builtin_bit_cast(bf16x8, d);
}

template <class EPI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_pairs_w1(const uint64_t* sig, const uint64_t* pairs,
                                                     const uint16_t* w1b, EPI E, uint32_t M,
                                                     uint32_t row_blocks) {
  __shared__ __attribute__((aligned(16))) uint16_t wt[2][kW1BN][kW1Pad];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, tid = threadIdx.x;
  const uint32_t xcd = blockIdx.x & 7u;
  const uint32_t rb = (blockIdx.x >> 3) * 2 + (xcd >> 2);
  if (rb >= row_blocks) return;  // padding blocks (the grid is a multiple of 8)
  const uint32_t n0 = (xcd & 3u) * kW1BN;
  const uint32_t m0 = rb * kW1BM + wv * 64;
  // this lane's two pair rows (tiles i = 0, 1) and their signature rows; a row
  // past M reads signature row 0 and is masked to zero
  const uint64_t* sa[2];
  const uint64_t* sb[2];
  uint64_t live[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const uint32_t r = m0 + 32 * i + (lane & 31);
    live[i] = r < M ? ~0ull : 0ull;
    const uint64_t pr = r < M ? pairs[r] : 0ull;
    sa[i] = sig + (pr >> 32) * kSigWords;
    sb[i] = sig + (pr & 0xFFFFFFFFu) * kSigWords;
  }
  // W1 loader: thread t copies row t / 2, k-half t % 2 (4 x 16 bytes) of a step
  const uint32_t lrow = tid >> 1, lk = (tid & 1) * 32;
  const uint16_t* wsrc = w1b + (uint64_t)(n0 + lrow) * kIn + lk;
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  u32x4 stage[4];
  auto load_w = [&](uint32_t k0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) stage[j] = *reinterpret_cast<const u32x4*>(wsrc + k0 + 8 * j);
  };
  auto store_w = [&](int buf) {
#pragma unroll
    for (int j = 0; j < 4; ++j) *reinterpret_cast<u32x4*>(&wt[buf][lrow][lk + 8 * j]) = stage[j];
  };
  // the step's pair word: k < 4096 -> XOR of the two signatures, else AND.
  // The raw words are loaded a step ahead and combined only when used, so
  // no wait for them (or for the W1 loads issued before them) falls inside
  // the step that issues them.
  auto combine = [&](int i, uint32_t step, uint64_t a, uint64_t b) -> uint64_t {
    return (step < 64 ? (a ^ b) : (a & b)) & live[i];
  };
  f32x16 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x16{0};

  constexpr uint32_t kSteps = kIn / kW1BK;  // 128
  load_w(0);
  store_w(0);
  uint64_t xw[2] = {combine(0, 0, sa[0][0], sb[0][0]), combine(1, 0, sa[1][0], sb[1][0])};
  __syncthreads();
  const uint32_t half = 8 * (lane >> 5);
  for (uint32_t step = 0; step < kSteps; ++step) {
    const int buf = step & 1;
    const bool more = step + 1 < kSteps;
    uint64_t na[2] = {0ull, 0ull}, nb[2] = {0ull, 0ull};
    if (more) {
      load_w((step + 1) * kW1BK);
      const uint32_t w = (step + 1) & 63u;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        na[i] = sa[i][w];
        nb[i] = sb[i][w];
      }
    }
    // keep the next step's loads ahead of this step's MFMAs (left alone, the
    // scheduler sinks them next to their use at the end of the step)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      bf16x8 a[2], b[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = expand_byte((uint32_t)(xw[i] >> (16 * q + half)) & 0xFFu);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        b[j] = *reinterpret_cast<const bf16x8*>(&wt[buf][32 * j + (lane & 31)][16 * q + half]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    // ... and their use after them (the MFMAs of the step issue first)
    __builtin_amdgcn_sched_barrier(0);
    if (more) {
      store_w(buf ^ 1);
#pragma unroll
      for (int i = 0; i < 2; ++i) xw[i] = combine(i, step + 1, na[i], nb[i]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint32_t m = m0 + 32 * i + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
        const uint32_t n = n0 + 32 * j + (lane & 31);
        if (m < M) E.store(m, n, acc[i][j][r]);
      }
}

template <class EPI>
hipError_t gemm_w1(const uint64_t* sig, const uint64_t* pairs, const uint16_t* w1b, EPI E,
                   uint32_t M, hipStream_t s) {
  const uint32_t row_blocks = (M + kW1BM - 1) / kW1BM;
  // 4 output quarters per row block; XCDs x and x + 4 take quarter x & 3
  const uint32_t grid = ((row_blocks + 1) / 2) * 8;
  hipLaunchKernelGGL((gemm_pairs_w1<EPI>), dim3(grid), dim3(256), 0, s, sig, pairs, w1b, E, M,
                     row_blocks);
  return hipGetLastError();
}

// ------------------------------------------------------------ small ops
// logit[m] = a2[m] . w3 + b3 (one wave per row, fixed-order reduction).
__global__ void head_forward(const float* a2, const float* w3, const float* b3, uint32_t M,
                             float* logit) {
  const uint32_t m = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (m >= M) return;
  float s = 0.f;
  for (int n = lane; n < kH2; n += 64) s += a2[(uint64_t)m * kH2 + n] * w3[n];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) logit[m] = s + b3[0];
}

// BCE-with-logits with positive weight p, mean over the batch:
// L = -(p y log s(z) + (1 - y) log(1 - s(z))), dL/dz = (s(z)(p y + 1 - y) - p y) / M.
// dz[m]; the input gradient of layer 2 (relu-masked) in fp32, bf16 and
// transposed bf16; the per-example loss terms.
__global__ void head_backward(const float* logit, const float* label, uint32_t M, float pw,
                              const float* w3, const float* a2, float* dz, float* lossv,
                              float* dh2_f, uint16_t* dh2, uint16_t* dh2_t, uint32_t ldt) {
  const uint32_t m = blockIdx.x;
  if (m >= M) return;
  const float z = logit[m], y = label[m];
  const float sg = 1.f / (1.f + expf(-z));
  const float g = (sg * (pw * y + 1.f - y) - pw * y) / (float)M;
  if (threadIdx.x == 0) {
    dz[m] = g;
    // log s(z) = -softplus(-z), log(1 - s(z)) = -softplus(z)
    const float sp_pos = fmaxf(z, 0.f) + log1pf(expf(-fabsf(z)));
    const float sp_neg = sp_pos - z;
    lossv[m] = pw * y * sp_neg + (1.f - y) * sp_pos;
  }
  for (uint32_t n = threadIdx.x; n < kH2; n += blockDim.x) {
    const float d = a2[(uint64_t)m * kH2 + n] > 0.f ? g * w3[n] : 0.f;
    dh2_f[(uint64_t)m * kH2 + n] = d;
    const uint16_t h = to_bf16(d);
    dh2[(uint64_t)m * kH2 + n] = h;
    dh2_t[(uint64_t)n * ldt + m] = h;
  }
}

// out[n] = sum_m X[m][n] (fixed order), optionally weighted by w[m].
__global__ void colsum(const float* X, const float* w, uint32_t M, uint32_t N, float* out) {
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (uint32_t m = 0; m < M; ++m) s += X[(uint64_t)m * N + n] * (w ? w[m] : 1.f);
  out[n] = s;
}

__global__ void vecsum(const float* x, uint32_t M, float* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float s = 0.f;
  for (uint32_t m = 0; m < M; ++m) s += x[m];
  out[0] = s;
}

__global__ void scale(float* x, uint32_t n, float a) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] *= a;
}

// Adam with bias correction on the FP32 master parameters.
__global__ void adam(float* p, const float* g, float* m1, float* m2, uint64_t n, float lr,
                     float b1, float b2, float eps, float c1, float c2) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  p[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

// BF16 working copies of W1, W2 and W2 transposed.
__global__ void refresh_bf16(const float* w1, const float* w2, uint16_t* w1b, uint16_t* w2b,
                             uint16_t* w2tb) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (uint64_t)kH1 * kIn) w1b[i] = to_bf16(w1[i]);
  if (i < (uint64_t)kH2 * kH1) {
    const uint32_t n = (uint32_t)(i / kH1), k = (uint32_t)(i % kH1);
    const uint16_t h = to_bf16(w2[i]);
    w2b[i] = h;
    w2tb[(uint64_t)k * kH2 + n] = h;
  }
}

inline uint32_t blocks(uint64_t n, uint32_t t = 256) { return (uint32_t)((n + t - 1) / t); }

}  // namespace mlp

using namespace mlp;

hipError_t mlp_refresh(MlpState& S, hipStream_t s) {
  hipLaunchKernelGGL(refresh_bf16, dim3(blocks((uint64_t)kH1 * kIn)), dim3(256), 0, s,
                     S.params + kOffW1, S.params + kOffW2, S.w1b, S.w2b, S.w2tb);
  return hipGetLastError();
}

// Forward of M pairs (M <= S.max_batch); with `train`, also the transposed
// layer-1 activations the weight gradient needs.
hipError_t mlp_forward(MlpState& S, const uint64_t* sig, const uint64_t* pairs, uint32_t M,
                       float* logit, bool train, hipStream_t s) {
  hipError_t e;
  PairRows X{sig, pairs, M};
  Dense W1{S.w1b, kIn, kH1};
  EpiHidden E1{S.params + kOffB1, S.a1, train ? S.a1t : nullptr, nullptr, kH1, S.max_batch};
  // layer 1: the LDS-staged kernel for batches that fill the chip (64 row
  // blocks x 4 quarters = one block per CU from 16,384 pairs), else the
  // direct-load one (training batches of a few hundred pairs)
  if (M >= 16384) {
    if ((e = gemm_w1(sig, pairs, S.w1b, E1, M, s))) return e;
  } else if ((e = gemm(X, W1, E1, M, kH1, kIn, s))) {
    return e;
  }
  Dense A1{S.a1, kH1, M};
  Dense W2{S.w2b, kH1, kH2};
  if (!train) {
    // scoring: layer 2 reduced against the head in its epilogue; the
    // per-group partials use the fp32 layer-2 buffer (needed only in training)
    if ((e = l2_head(A1, W2, S.params + kOffB2, S.params + kOffW3, S.a2, M, s))) return e;
    hipLaunchKernelGGL(head_sum, dim3(blocks(M)), dim3(256), 0, s, S.a2, S.params + kOffB3, M,
                       logit);
    return hipGetLastError();
  }
  EpiHidden E2{S.params + kOffB2, S.a2b, nullptr, S.a2, kH2, 0};
  if ((e = gemm(A1, W2, E2, M, kH2, kH1, s))) return e;
  hipLaunchKernelGGL(head_forward, dim3(blocks(M, 4)), dim3(256), 0, s, S.a2,
                     S.params + kOffW3, S.params + kOffB3, M, logit);
  return hipGetLastError();
}

// Loss and all parameter gradients of one batch into S.grads (no update).
hipError_t mlp_backward(MlpState& S, const uint64_t* sig, const uint64_t* pairs,
                        const float* label, uint32_t M, float pos_weight, float* loss,
                        hipStream_t s) {
  hipError_t e;
  if ((e = mlp_forward(S, sig, pairs, M, S.logit, true, s))) return e;
  float* G = S.grads;
  hipLaunchKernelGGL(head_backward, dim3(M), dim3(256), 0, s, S.logit, label, M, pos_weight,
                     S.params + kOffW3, S.a2, S.dz, S.lossv, S.dh2f, S.dh2, S.dh2t, S.max_batch);
  // head: dw3 = a2^T dz, db3 = sum dz, loss = sum of terms / M
  hipLaunchKernelGGL(colsum, dim3(blocks(kH2)), dim3(256), 0, s, S.a2, S.dz, M, kH2, G + kOffW3);
  hipLaunchKernelGGL(vecsum, dim3(1), dim3(64), 0, s, S.dz, M, G + kOffB3);
  hipLaunchKernelGGL(vecsum, dim3(1), dim3(64), 0, s, S.lossv, M, loss);
  hipLaunchKernelGGL(scale, dim3(1), dim3(64), 0, s, loss, 1u, 1.f / (float)M);
  // layer 2: db2 = colsum dh2, dW2[n][k] = sum_m dh2[m][n] a1[m][k]
  hipLaunchKernelGGL(colsum, dim3(blocks(kH2)), dim3(256), 0, s, S.dh2f, nullptr, M, kH2,
                     G + kOffB2);
  {
    Dense A{S.dh2t, S.max_batch, kH2};
    Dense B{S.a1t, S.max_batch, kH1};
    EpiStore E{G + kOffW2, kH1};
    if ((e = gemm(A, B, E, kH2, kH1, M, s))) return e;
  }
  // layer 1 input gradient: dA1[m][k] = sum_n dh2[m][n] W2[n][k], relu mask
  {
    Dense A{S.dh2, kH2, M};
    Dense B{S.w2tb, kH2, kH1};
    EpiReluGrad E{S.a1, S.dh1f, S.dh1t, kH1, S.max_batch};
    if ((e = gemm(A, B, E, M, kH1, kH2, s))) return e;
  }
  hipLaunchKernelGGL(colsum, dim3(blocks(kH1)), dim3(256), 0, s, S.dh1f, nullptr, M, kH1,
                     G + kOffB1);
  // dW1[n][f] = sum_m dh1[m][n] x[m][f]
  {
    Dense A{S.dh1t, S.max_batch, kH1};
    PairCols B{sig, pairs, M};
    EpiStore E{G + kOffW1, kIn};
    if ((e = gemm(A, B, E, kH1, kIn, M, s))) return e;
  }
  return hipGetLastError();
}

hipError_t mlp_adam(MlpState& S, float lr, float b1, float b2, float eps, hipStream_t s) {
  S.step += 1;
  const float c1 = 1.f - powf(b1, (float)S.step), c2 = 1.f - powf(b2, (float)S.step);
  hipLaunchKernelGGL(adam, dim3(blocks(kParams)), dim3(256), 0, s, S.params, S.grads, S.m1, S.m2,
                     (uint64_t)kParams, lr, b1, b2, eps, c1, c2);
  hipError_t e = hipGetLastError();
  if (e) return e;
  return mlp_refresh(S, s);
}

}  // namespace kripke
