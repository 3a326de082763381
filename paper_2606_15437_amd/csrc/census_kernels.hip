// Census and split kernels for gfx950 (MI355X).
//
// Representation (Section 3): a truth set over the n worlds of one model is a
// bitmask; here it is bit-sliced across valuations instead: for each world w
// a 32-bit word holds the truth of the subformula at w under 32 consecutive
// valuations.  Boolean connectives are then one bitwise instruction per world
// for 32 models, and Lemma 1's modal identities become, per world w,
//   DIA t : OR over v of (R(w,v) & t_v),   BOX t : AND over v of (~R(w,v) | t_v),
// where R(w,v) is an all-ones/all-zeros word.  All of this is integer VALU
// work; there is no floating point and no matrix-core use in the evaluator.
//
// Valuation index bits 0..4 live inside the word, so p_i at world w is a
// constant pattern when i*n + w < 5 (0xAAAAAAAA, 0xCCCCCCCC, ...); higher
// valuation bits come from the lane's word index.
//
// Each wavefront interprets one formula at a time.  The compiled program is
// staged in LDS and read as wave-uniform bytes, so dispatch is scalar and
// the 64 lanes evaluate 64 (frame, valuation-word) units in lock step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>

#include "kripke_internal.h"
#include "census_kernels.h"

namespace kripke {

// Bit j of pattern(b) is bit b of j: valuation bit b < 5 inside a word.
__host__ __device__ constexpr uint32_t pattern(int b) {
  return b == 0 ? 0xAAAAAAAAu : b == 1 ? 0xCCCCCCCCu : b == 2 ? 0xF0F0F0F0u
       : b == 3 ? 0xFF00FF00u : 0xFFFF0000u;
}

__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int lane) {
  uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, lane);
  uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

// Reflexive frames on n worlds, enumerated in increasing index order:
// position j deposits its bits into the off-diagonal positions.
__host__ __device__ __forceinline__ uint64_t t_frame(uint64_t j, int n) {
  uint64_t full = (1ull << n) - 1, f = 0;
  for (int w = 0; w < n; ++w) f |= 1ull << (w * n + w);
  for (int k = 0; k + 1 < n; ++k) f |= ((j >> (k * n)) & full) << (k * (n + 1) + 1);
  return f;
}

// --------------------------------------------------------------- evaluator
template <int N, int NV>
struct Regs {
  static constexpr int V = N * NV;
  static constexpr int kVat = V > 5 ? V - 5 : 1;
  uint32_t R[N][N];      // all-ones / all-zeros relation words
  uint32_t vat[kVat];    // p_i at w for valuation bits >= 5 (per lane)
  uint32_t acc[N];       // the accumulator truth set
  uint32_t stk[kMaxSlots][N];
};

template <int N, int NV>
__device__ __forceinline__ uint32_t var_word(const Regs<N, NV>& r, int i, int w) {
  const int b = i * N + w;
  if (b < 5) return pattern(b);
  return r.vat[b - 5];
}

template <int N, int NV, int L>
__device__ __forceinline__ uint32_t leaf_word(const Regs<N, NV>& r, int w) {
  if constexpr (L < 4) {
    return var_word<N, NV>(r, L, w);
  } else if constexpr (L < 8) {
    return ~var_word<N, NV>(r, L - 4, w);
  } else if constexpr (L == L_SUCC || L == L_DEAD) {
    uint32_t s = 0;
#pragma unroll
    for (int v = 0; v < N; ++v) s |= r.R[w][v];
    return L == L_SUCC ? s : ~s;
  } else if constexpr (L == L_TOP) {
    return ~0u;
  } else {
    return 0u;
  }
}

template <int N, int NV, int L>
__device__ __forceinline__ void op_load(Regs<N, NV>& r) {
#pragma unroll
  for (int w = 0; w < N; ++w) r.acc[w] = leaf_word<N, NV, L>(r, w);
}

template <int N, int NV, int L>
__device__ __forceinline__ void op_and_l(Regs<N, NV>& r) {
#pragma unroll
  for (int w = 0; w < N; ++w) r.acc[w] &= leaf_word<N, NV, L>(r, w);
}

template <int N, int NV, int L>
__device__ __forceinline__ void op_or_l(Regs<N, NV>& r) {
#pragma unroll
  for (int w = 0; w < N; ++w) r.acc[w] |= leaf_word<N, NV, L>(r, w);
}

template <int N, int NV, int L>
__device__ __forceinline__ void op_iff_l(Regs<N, NV>& r) {
#pragma unroll
  for (int w = 0; w < N; ++w) r.acc[w] = ~(r.acc[w] ^ leaf_word<N, NV, L>(r, w));
}

template <int N, int NV>
__device__ __forceinline__ void op_dia(Regs<N, NV>& r) {
  uint32_t t[N];
#pragma unroll
  for (int w = 0; w < N; ++w) {
    uint32_t s = 0;
#pragma unroll
    for (int v = 0; v < N; ++v) s |= r.R[w][v] & r.acc[v];
    t[w] = s;
  }
#pragma unroll
  for (int w = 0; w < N; ++w) r.acc[w] = t[w];
}

template <int N, int NV>
__device__ __forceinline__ void op_box(Regs<N, NV>& r) {
  uint32_t t[N];
#pragma unroll
  for (int w = 0; w < N; ++w) {
    uint32_t s = ~0u;
#pragma unroll
    for (int v = 0; v < N; ++v) s &= ~r.R[w][v] | r.acc[v];
    t[w] = s;
  }
#pragma unroll
  for (int w = 0; w < N; ++w) r.acc[w] = t[w];
}

// DIA/BOX applied directly to a variable literal (a superinstruction).
template <int N, int NV, bool DIA, int L>
__device__ __forceinline__ void op_modal_leaf(Regs<N, NV>& r) {
#pragma unroll
  for (int v = 0; v < N; ++v) r.acc[v] = leaf_word<N, NV, L>(r, v);
  if constexpr (DIA) op_dia<N, NV>(r);
  else op_box<N, NV>(r);
}

template <int N, int NV, int D>
__device__ __forceinline__ void op_save(Regs<N, NV>& r) {
#pragma unroll
  for (int w = 0; w < N; ++w) r.stk[D][w] = r.acc[w];
}

template <int N, int NV, int D, int OP>
__device__ __forceinline__ void op_comb(Regs<N, NV>& r) {
#pragma unroll
  for (int w = 0; w < N; ++w) {
    if constexpr (OP == 0) r.acc[w] &= r.stk[D][w];
    else if constexpr (OP == 1) r.acc[w] |= r.stk[D][w];
    else r.acc[w] = ~(r.acc[w] ^ r.stk[D][w]);
  }
}

#define KR_LEAF10(BASE, FN)                                                        \
  case BASE + 0: FN(0); break; case BASE + 1: FN(1); break; case BASE + 2: FN(2); break; \
  case BASE + 3: FN(3); break; case BASE + 4: FN(4); break; case BASE + 5: FN(5); break; \
  case BASE + 6: FN(6); break; case BASE + 7: FN(7); break; case BASE + 8: FN(8); break; \
  case BASE + 9: FN(9); break;
#define KR_SLOT8(BASE, FN)                                                         \
  case BASE + 0: FN(0); break; case BASE + 1: FN(1); break; case BASE + 2: FN(2); break; \
  case BASE + 3: FN(3); break; case BASE + 4: FN(4); break; case BASE + 5: FN(5); break; \
  case BASE + 6: FN(6); break; case BASE + 7: FN(7); break;

// Run the wave's staged program on the current registers; result in r.acc.
template <int N, int NV>
__device__ __forceinline__ void interpret(Regs<N, NV>& r, const uint32_t* prog) {
  uint32_t cur = 0;
  for (int pc = 0;; ++pc) {
    if ((pc & 3) == 0) cur = __builtin_amdgcn_readfirstlane(prog[pc >> 2]);
    const uint32_t op = (cur >> ((pc & 3) * 8)) & 0xffu;
    if (op == U_END) break;
#define F_LOAD(L) op_load<N, NV, L>(r)
#define F_AND(L) op_and_l<N, NV, L>(r)
#define F_OR(L) op_or_l<N, NV, L>(r)
#define F_IFF(L) op_iff_l<N, NV, L>(r)
#define F_SAVE(D) op_save<N, NV, D>(r)
#define F_ANDS(D) op_comb<N, NV, D, 0>(r)
#define F_ORS(D) op_comb<N, NV, D, 1>(r)
#define F_IFFS(D) op_comb<N, NV, D, 2>(r)
#define F_DIAL(L) op_modal_leaf<N, NV, true, L>(r)
#define F_BOXL(L) op_modal_leaf<N, NV, false, L>(r)
    switch (op) {
      KR_LEAF10(U_LOAD, F_LOAD)
      case U_LOAD + L_TOP: F_LOAD(L_TOP); break;
      case U_LOAD + L_BOT: F_LOAD(L_BOT); break;
      KR_LEAF10(U_AND_L, F_AND)
      KR_LEAF10(U_OR_L, F_OR)
      KR_LEAF10(U_IFF_L, F_IFF)
      case U_BOX: op_box<N, NV>(r); break;
      case U_DIA: op_dia<N, NV>(r); break;
      KR_SLOT8(U_SAVE, F_SAVE)
      KR_SLOT8(U_AND_S, F_ANDS)
      KR_SLOT8(U_OR_S, F_ORS)
      KR_SLOT8(U_IFF_S, F_IFFS)
      KR_SLOT8(U_DIA_L, F_DIAL)
      KR_SLOT8(U_BOX_L, F_BOXL)
      case U_MM + 0: op_box<N, NV>(r); op_box<N, NV>(r); break;
      case U_MM + 1: op_box<N, NV>(r); op_dia<N, NV>(r); break;
      case U_MM + 2: op_dia<N, NV>(r); op_box<N, NV>(r); break;
      case U_MM + 3: op_dia<N, NV>(r); op_dia<N, NV>(r); break;
      default: break;
    }
#undef F_LOAD
#undef F_AND
#undef F_OR
#undef F_IFF
#undef F_SAVE
#undef F_ANDS
#undef F_ORS
#undef F_IFFS
#undef F_DIAL
#undef F_BOXL
  }
}

// --------------------------------------------------------------- census
// One wavefront pops work items (formula, range of 64-unit blocks) from a
// global counter until the queue is empty.  A unit is one (frame position,
// 32-valuation word) pair; lanes take consecutive units, so within a block
// the lowest failing lane holds the lexicographically least countermodel.
template <int N, int NV>
__global__ __launch_bounds__(256) void census_generic(CensusArgs a) {
  constexpr int V = N * NV;
  constexpr int WLOG = V > 5 ? V - 5 : 0;
  __shared__ uint32_t sprog[4][kMaxMicro / 4 + 4];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  uint32_t* prog = sprog[wv];
  const uint32_t inword = V >= 5 ? 0xFFFFFFFFu : ((1u << (1u << V)) - 1u);
  const uint64_t units = a.npos << WLOG;
  const uint64_t nblocks = (units + 63) >> 6;

  for (;;) {
    uint64_t item = 0;
    if (lane == 0) item = atomicAdd(a.queue, 1ull);
    item = readlane64(item, 0);
    if (item >= a.total_items) break;
    const uint32_t fslot = (uint32_t)(item / a.items_per_formula);
    const uint32_t f = a.order[fslot];
    const uint64_t b0 = (item % a.items_per_formula) * a.blocks_per_item;
    const uint64_t b1 = b0 + a.blocks_per_item < nblocks ? b0 + a.blocks_per_item : nblocks;
    unsigned long long* key_out = a.out_key + (uint64_t)f * a.out_stride;

    // DECIDE: skip the item if an earlier countermodel is already known.
    if (a.decide) {
      uint64_t first_pos = (b0 << 6) >> WLOG;
      uint64_t first_frame;
      if (a.key_pos) first_frame = a.pos_begin + first_pos;
      else if (a.mode == M_RANGE_K) first_frame = a.pos_begin + first_pos;
      else if (a.mode == M_RANGE_T) first_frame = N * N <= 64 ? t_frame(a.pos_begin + first_pos, N) : 0;
      else first_frame = a.list_idx[a.pos_begin + first_pos];
      uint64_t known = __hip_atomic_load(key_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      known = uniform64(known);
      if (known != ~0ull && (known >> (V + 4)) < first_frame) continue;
    }

    // stage the compiled program of formula f in this wave's LDS slice
    const uint32_t p0 = a.uoff[f] >> 2, pw = (a.uoff[f + 1] >> 2) - p0;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.ucode) + p0;
    for (uint32_t i = lane; i < pw; i += 64) prog[i] = src[i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    uint32_t cnt = 0;
    uint64_t key = ~0ull;
    Regs<N, NV> r;
    for (uint64_t blk = b0; blk < b1; ++blk) {
      const uint64_t u = (blk << 6) + lane;
      const uint64_t pos = u >> WLOG;
      const uint32_t word = (uint32_t)(u & ((1ull << WLOG) - 1));
      const bool valid = pos < a.npos;
      const uint64_t p = a.pos_begin + (valid ? pos : 0);
      uint64_t frame = 0;
      if (a.mode == M_LIST_SUCC) {
        const uint32_t* s = a.list_succ + p * N;
#pragma unroll
        for (int w = 0; w < N; ++w) {
          const uint32_t sw = s[w];
#pragma unroll
          for (int v = 0; v < N; ++v) r.R[w][v] = 0u - ((sw >> v) & 1u);
        }
        frame = p;
      } else if constexpr (N * N <= 64) {
        // frame indices exist only while the relation fits 64 bits
        if (a.mode == M_RANGE_K) frame = p;
        else if (a.mode == M_RANGE_T) frame = t_frame(p, N);
        else frame = a.list_idx[p];
#pragma unroll
        for (int w = 0; w < N; ++w)
#pragma unroll
          for (int v = 0; v < N; ++v) r.R[w][v] = 0u - (uint32_t)((frame >> (w * N + v)) & 1u);
      }
#pragma unroll
      for (int i = 0; i < Regs<N, NV>::kVat; ++i) r.vat[i] = 0u - ((word >> i) & 1u);

      interpret<N, NV>(r, prog);

      uint32_t all = ~0u;
#pragma unroll
      for (int w = 0; w < N; ++w) all &= r.acc[w];
      const uint32_t fail = valid ? (~all & inword) : 0u;
      cnt += __builtin_popcount(fail);
      if (key == ~0ull) {
        const uint64_t bal = __ballot(fail != 0);
        if (bal) {
          const int fl = __builtin_ctzll(bal);
          const uint32_t j = __builtin_ctz(fail | 0x80000000u);
          uint32_t world = 0;
#pragma unroll
          for (int w = N - 1; w >= 0; --w)
            if (!((r.acc[w] >> j) & 1u)) world = w;
          const uint64_t fld = a.key_pos ? p : frame;
          const uint64_t lk = (fld << (V + 4)) | ((uint64_t)((word << 5) | j) << 4) | world;
          key = readlane64(lk, fl);
          if (a.decide) break;
        }
      }
    }
    // wave reduction, then one atomic per counter per wave and work item
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    if (lane == 0) {
      if (key != ~0ull) atomicMin(key_out, (unsigned long long)key);
      if (cnt && a.out_cnt) atomicAdd(a.out_cnt + (uint64_t)f * a.out_stride, (unsigned long long)cnt);
    }
  }
}

// ----------------------------------------------------------- signatures
// Truth bits of formulas at sampled pointed models (n, frame, valuation,
// world), 64 samples per wavefront: each lane evaluates its sample's frame
// on the 32-valuation word holding the sample's valuation and keeps one bit;
// a ballot packs the 64 bits into one word of the signature.
template <int N, int NV>
__global__ __launch_bounds__(256) void signature_kernel(SigArgs a) {
  constexpr int V = N * NV;
  __shared__ uint32_t sprog[4][kMaxMicro / 4 + 4];
  const int lane = threadIdx.x & 63;
  uint32_t* prog = sprog[threadIdx.x >> 6];
  const uint64_t total = (uint64_t)a.nformulas * a.ngroups;
  const uint64_t wave = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint64_t stride = (uint64_t)gridDim.x * 4;
  uint32_t staged = ~0u;
  Regs<N, NV> r;
  for (uint64_t item = wave; item < total; item += stride) {
    const uint32_t f = (uint32_t)(item / a.ngroups);
    const uint32_t g = a.groups[item % a.ngroups];
    if (f != staged) {
      const uint32_t p0 = a.uoff[f] >> 2, pw = (a.uoff[f + 1] >> 2) - p0;
      const uint32_t* src = reinterpret_cast<const uint32_t*>(a.ucode) + p0;
      __builtin_amdgcn_wave_barrier();
      for (uint32_t i = lane; i < pw; i += 64) prog[i] = src[i];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      staged = f;
    }
    const uint64_t smp = a.samples[(uint64_t)g * 64 + lane];
    const uint64_t frame = (smp >> 24) & 0xFFFFFFFFFull;
    const uint32_t val = (uint32_t)(smp >> 4) & 0xFFFFFu;
    const uint32_t world = (uint32_t)(smp & 15u);
#pragma unroll
    for (int w = 0; w < N; ++w)
#pragma unroll
      for (int v = 0; v < N; ++v) r.R[w][v] = 0u - (uint32_t)((frame >> (w * N + v)) & 1u);
    const uint32_t word = V > 5 ? (val >> 5) : 0u;
#pragma unroll
    for (int i = 0; i < Regs<N, NV>::kVat; ++i) r.vat[i] = 0u - ((word >> i) & 1u);
    interpret<N, NV>(r, prog);
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < N; ++w)
      if ((uint32_t)w == world) t = r.acc[w];
    const uint64_t bits = __ballot(((t >> (val & 31u)) & 1u) != 0);
    if (lane == 0) a.sig[(uint64_t)f * a.words + g] = bits;
  }
}

// ------------------------------------------------------- helper kernels
__global__ void init_results(unsigned long long* key, unsigned long long* cnt, uint32_t stride,
                             uint32_t count, unsigned long long* queue) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    key[(uint64_t)i * stride] = ~0ull;
    if (cnt) cnt[(uint64_t)i * stride] = 0ull;
  }
  if (i == 0 && queue) *queue = 0ull;
}

// Class level of every frame on n worlds: 0 K only, 1 reflexive, 2 reflexive
// and transitive (S4), 3 equivalence relation (S5).
__device__ __forceinline__ int class_level(uint64_t f, int n) {
  const uint32_t full = (1u << n) - 1u;
  uint32_t succ[8];
  for (int w = 0; w < n; ++w) succ[w] = (uint32_t)(f >> (w * n)) & full;
  for (int w = 0; w < n; ++w)
    if (!((succ[w] >> w) & 1u)) return 0;
  for (int w = 0; w < n; ++w)
    for (int v = 0; v < n; ++v)
      if (((succ[w] >> v) & 1u) && (succ[v] & ~succ[w])) return 1;
  for (int w = 0; w < n; ++w)
    for (int v = 0; v < n; ++v)
      if (((succ[w] >> v) & 1u) != ((succ[v] >> w) & 1u)) return 2;
  return 3;
}

// Ordered stream compaction of the frames of one class, in three passes:
// per-256-frame counts, an exclusive scan of the counts, and the scatter.
__global__ void class_count(int n, int level, uint64_t nframes, uint32_t* counts) {
  const uint64_t f = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const bool in = f < nframes && class_level(f, n) >= level;
  const uint64_t bal = __ballot(in);
  __shared__ uint32_t part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = __builtin_popcountll(bal);
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

__global__ void class_scan(uint32_t* counts, uint32_t nblocks, uint64_t* total) {
  // single block of 1024 threads: each thread scans a contiguous chunk
  __shared__ uint64_t sums[1024];
  const uint32_t t = threadIdx.x;
  const uint32_t per = (nblocks + 1023) / 1024;
  const uint32_t lo = t * per, hi = lo + per < nblocks ? lo + per : nblocks;
  uint64_t s = 0;
  for (uint32_t i = lo; i < hi; ++i) s += counts[i];
  sums[t] = s;
  __syncthreads();
  if (t == 0) {
    uint64_t run = 0;
    for (int i = 0; i < 1024; ++i) {
      uint64_t x = sums[i];
      sums[i] = run;
      run += x;
    }
    *total = run;
  }
  __syncthreads();
  uint64_t run = sums[t];
  for (uint32_t i = lo; i < hi; ++i) {
    uint32_t x = counts[i];
    counts[i] = (uint32_t)run;
    run += x;
  }
}

__global__ void class_scatter(int n, int level, uint64_t nframes, const uint32_t* offsets,
                              uint64_t* list) {
  const uint64_t f = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const bool in = f < nframes && class_level(f, n) >= level;
  const uint64_t bal = __ballot(in);
  __shared__ uint32_t part[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) part[wv] = __builtin_popcountll(bal);
  __syncthreads();
  uint32_t base = offsets[blockIdx.x];
  for (int i = 0; i < wv; ++i) base += part[i];
  const uint32_t rank = __builtin_popcountll(bal & ((1ull << lane) - 1ull));
  if (in) list[base + rank] = f;
}

// ------------------------------------------------------------ dispatch
hipError_t launch_signatures(const SigArgs& a, int n, int nvars, hipStream_t s) {
  const uint64_t total = (uint64_t)a.nformulas * a.ngroups;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((total + 3) / 4, 256u * 64u);
  if (total == 0) return hipSuccess;
#define KR_SIG(N, NV)                                                                     \
  if (n == N && nvars == NV) {                                                           \
    hipLaunchKernelGGL((signature_kernel<N, NV>), dim3(grid), dim3(256), 0, s, a);        \
    return hipGetLastError();                                                             \
  }
  KR_SIG(1, 0) KR_SIG(1, 1) KR_SIG(1, 2) KR_SIG(1, 3) KR_SIG(1, 4)
  KR_SIG(2, 0) KR_SIG(2, 1) KR_SIG(2, 2) KR_SIG(2, 3) KR_SIG(2, 4)
  KR_SIG(3, 0) KR_SIG(3, 1) KR_SIG(3, 2) KR_SIG(3, 3) KR_SIG(3, 4)
#undef KR_SIG
  return hipErrorInvalidValue;
}

template <int N, int NV>
static hipError_t launch_one(const CensusArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((census_generic<N, NV>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Resident blocks per CU, queried once per kernel (the query costs about a
// millisecond of host time, which per-formula launch loops would pay each time).
template <int N, int NV>
static int occupancy_one() {
  static std::atomic<int> cached{0};
  int blocks = cached.load(std::memory_order_relaxed);
  if (blocks > 0) return blocks;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, census_generic<N, NV>, 256, 0) !=
          hipSuccess ||
      blocks <= 0)
    return 1;
  cached.store(blocks, std::memory_order_relaxed);
  return blocks;
}

#define KR_NV_TABLE(N) {&launch_one<N, 0>, &launch_one<N, 1>, &launch_one<N, 2>, \
                        &launch_one<N, 3>, &launch_one<N, 4>}
#define KR_OCC_TABLE(N) {&occupancy_one<N, 0>, &occupancy_one<N, 1>, &occupancy_one<N, 2>, \
                         &occupancy_one<N, 3>, &occupancy_one<N, 4>}

using LaunchFn = hipError_t (*)(const CensusArgs&, int, hipStream_t);
using OccFn = int (*)();

// 9 and 10 worlds: frame lists only, at most one variable (template frames for
// constant and one-variable formulas)
static const LaunchFn kLaunch[10][5] = {
    KR_NV_TABLE(1), KR_NV_TABLE(2), KR_NV_TABLE(3), KR_NV_TABLE(4), KR_NV_TABLE(5),
    KR_NV_TABLE(6),
    {&launch_one<7, 0>, &launch_one<7, 1>, &launch_one<7, 2>, &launch_one<7, 3>, nullptr},
    {&launch_one<8, 0>, &launch_one<8, 1>, &launch_one<8, 2>, &launch_one<8, 3>, nullptr},
    {&launch_one<9, 0>, &launch_one<9, 1>, nullptr, nullptr, nullptr},
    {&launch_one<10, 0>, &launch_one<10, 1>, nullptr, nullptr, nullptr}};
static const OccFn kOcc[10][5] = {
    KR_OCC_TABLE(1), KR_OCC_TABLE(2), KR_OCC_TABLE(3), KR_OCC_TABLE(4), KR_OCC_TABLE(5),
    KR_OCC_TABLE(6),
    {&occupancy_one<7, 0>, &occupancy_one<7, 1>, &occupancy_one<7, 2>, &occupancy_one<7, 3>,
     nullptr},
    {&occupancy_one<8, 0>, &occupancy_one<8, 1>, &occupancy_one<8, 2>, &occupancy_one<8, 3>,
     nullptr},
    {&occupancy_one<9, 0>, &occupancy_one<9, 1>, nullptr, nullptr, nullptr},
    {&occupancy_one<10, 0>, &occupancy_one<10, 1>, nullptr, nullptr, nullptr}};

hipError_t launch_census(const CensusArgs& a, int n, int nvars, int grid, hipStream_t s) {
  if (n < 1 || n > 10 || nvars < 0 || nvars > 4 || !kLaunch[n - 1][nvars])
    return hipErrorInvalidValue;
  return kLaunch[n - 1][nvars](a, grid, s);
}

int census_blocks_per_cu(int n, int nvars) {
  if (n < 1 || n > 10 || nvars < 0 || nvars > 4 || !kOcc[n - 1][nvars]) return 1;
  return kOcc[n - 1][nvars]();
}

uint64_t t_frame_host(uint64_t j, int n) { return t_frame(j, n); }

hipError_t launch_init(unsigned long long* key, unsigned long long* cnt, uint32_t stride,
                       uint32_t count, unsigned long long* queue, hipStream_t s) {
  const uint32_t blocks = (count + 255) / 256 ? (count + 255) / 256 : 1;
  hipLaunchKernelGGL(init_results, dim3(blocks), dim3(256), 0, s, key, cnt, stride, count, queue);
  return hipGetLastError();
}

__global__ void fill_rows(uint32_t* rows, uint64_t words, const uint32_t* value, uint32_t nrows) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words * nrows) rows[i] = value[i / words];
}

hipError_t launch_fill_rows(uint32_t* rows, uint64_t words, const uint32_t* value, uint32_t nrows,
                            hipStream_t s) {
  const uint64_t total = words * nrows;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_rows, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, s, rows,
                     words, value, nrows);
  return hipGetLastError();
}

hipError_t launch_class_list(int n, int level, uint32_t* counts, uint64_t* total, uint64_t* list,
                             hipStream_t s) {
  const uint64_t nframes = 1ull << (n * n);
  const uint32_t nblocks = (uint32_t)((nframes + 255) / 256);
  hipLaunchKernelGGL(class_count, dim3(nblocks), dim3(256), 0, s, n, level, nframes, counts);
  hipLaunchKernelGGL(class_scan, dim3(1), dim3(1024), 0, s, counts, nblocks, total);
  if (list)
    hipLaunchKernelGGL(class_scatter, dim3(nblocks), dim3(256), 0, s, n, level, nframes, counts,
                       list);
  return hipGetLastError();
}

}  // namespace kripke
