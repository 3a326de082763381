// Fast census kernel for gfx950: wave-uniform frames.
//
// The generic kernel gives every lane its own frame, so every relation word
// R(w,v) is a vector register rebuilt per block.  Here a wavefront works on
// a block of 2^(LF+LS) consecutive frames (in class enumeration order):
//   - the 5 in-word bits and the low lane bits index valuations, exactly as
//     in the generic kernel (all valuations of a frame sit in one wave when
//     n*k <= 11);
//   - the remaining LF lane bits index LF frame positions (per-lane relation
//     words, fixed for the whole kernel);
//   - LS "set" bits index the next frame positions: every lane evaluates the
//     formula on 2^LS frames at once, and the relation words of those
//     positions are compile-time constants per set;
//   - all other relation bits are shared by the whole block: scalar
//     registers, decoded once per block by the scalar unit.
// So Lemma 1's DIA/BOX cost one VALU op per (world, successor) term with a
// scalar operand, constant terms fold away, and one scalar interpreter
// dispatch drives 2^LS sets of VALU work.
//
// Frame enumeration: mode K scans raw frame indices; mode T scans reflexive
// frames in index order (positions deposit into the off-diagonal bits).  In
// mode K with `fused`, each frame also reduces into the classes T, S4 and S5
// it belongs to (a precomputed 2-bit class level per frame), so one pass over
// the K frames yields the census of all four classes.
//
// Mode LIST (split search over a caller's frame list, n * nvars >= 11): a
// block is ONE list frame, so every relation word is wave-uniform and comes
// from the frame's successor rows; the set bits then index valuation bits
// 11 .. 11+LS-1 (between the lane bits and the chunk loop) instead of frames.
// Where a frame has only 2^12 valuations (six worlds, two variables) a wave
// would carry just two sets per interpreter dispatch; mode LIST2 instead puts
// two list frames in a block, one per half-wave (lane bit 5 is a frame bit,
// the relation words are per-lane values), with four sets over valuation bits
// 10 and 11, so each dispatch and each relation decode serves two frames.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>

#include "census_kernels.h"
#include "kripke_internal.h"

namespace kripke {
namespace {

__host__ __device__ constexpr uint32_t pattern(int b) {
  return b == 0 ? 0xAAAAAAAAu : b == 1 ? 0xCCCCCCCCu : b == 2 ? 0xF0F0F0F0u
       : b == 3 ? 0xFF00FF00u : 0xFFFF0000u;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int lane) {
  uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, lane);
  uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

__host__ __device__ __forceinline__ uint64_t refl_frame(uint64_t j, int n) {
  uint64_t full = (1ull << n) - 1, f = 0;
  for (int w = 0; w < n; ++w) f |= 1ull << (w * n + w);
  for (int k = 0; k + 1 < n; ++k) f |= ((j >> (k * n)) & full) << (k * (n + 1) + 1);
  return f;
}

enum Role { R_UNIFORM = 0, R_LANE = 1, R_SET = 2, R_ONE = 3 };

template <int N, int MODE>
__host__ __device__ constexpr int free_rank(int p) {
  // rank of position p among the enumerated (free) positions
  return MODE == 0 ? p : p - p / (N + 1) - 1;
}

template <int N, int MODE, int LF, int LS>
__host__ __device__ constexpr int role(int p) {
  if (MODE >= 2) return R_UNIFORM;
  if (MODE == 1 && p % (N + 1) == 0) return R_ONE;
  const int r = free_rank<N, MODE>(p);
  return r < LF ? R_LANE : r < LF + LS ? R_SET : R_UNIFORM;
}

template <int N, int MODE>
__host__ __device__ constexpr int role_idx(int p, int LF) {
  const int r = free_rank<N, MODE>(p);
  return r < LF ? r : r - LF;
}

// List-mode relation rows held in vector registers, per variant: as many as
// fit four waves per SIMD (at most 128 VGPRs).  At n = 7 and 8 with four sets
// the kernel also keeps two sets of its register stack slot in LDS and has no
// whole LDS slot, which buys more rows (measured on the split search: at
// n = 8, 483 ms with three rows and an LDS slot, 459 ms with five; at n = 7,
// 468 ms with one row, two register slots and an LDS slot, 410 ms with six).
__host__ __device__ constexpr int list_rows(int n, int ls) {
  return n == 6 ? 6 : n == 7 ? (ls == 0 ? 7 : 6) : (ls == 0 ? 6 : 5);
}
__host__ __device__ constexpr bool list_four_sets(bool list, int n, int ls) {
  return list && n >= 7 && ls == 2;
}

template <int N, int NV, int LS, int MODE>
struct Geo {
  static constexpr bool LIST = MODE >= 2;
  // two list frames per block, one per half-wave (their relation words are
  // per-lane values), for lists whose frames have too few valuations to fill
  // a wave with several sets
  static constexpr bool LIST2 = MODE == 3;
  static constexpr int V = N * NV;
  static constexpr int LV = LIST2 ? 5 : V >= 11 ? 6 : (V > 5 ? V - 5 : 0);  // lane valuation bits
  static constexpr int LF = 6 - LV;                              // lane frame bits
  static constexpr int S = 1 << LS;                              // sets per lane
  static constexpr int SV = LIST ? LS : 0;                       // set bits that are valuation bits
  static constexpr int B = LIST2 ? 1 : LIST ? 0 : LF + LS;       // log2 frames per block
  static constexpr int CHB = V > 5 + LV + SV ? V - 5 - LV - SV : 0;  // valuation chunk bits
  // stack slots in registers (one at the seven- and eight-world four-set list
  // variants)
  static constexpr int DS =
      LS == 0 ? 4 : (LS <= 2 && !list_four_sets(LIST, N, LS) && !LIST2) ? 2 : 1;
  // + slots held wholly in LDS; none at LS = 3 (40 KB per block would cap
  // residency at three blocks per CU) nor in the seven- and eight-world
  // four-set list variants (their LDS stack sets already take 14-16 KB per
  // block): programs needing more slots run in a narrower tier
  static constexpr int LDS_SLOTS = LS >= 3 || list_four_sets(LIST, N, LS) ? 0 : 1;
  // Block-uniform relation words held in vector registers, by rows of the
  // relation: on gfx950 a VALU instruction with a scalar operand issues at
  // half the rate of one with vector operands only, and the modal terms are
  // most of the work.  Census modes hold every row; list mode (n^2 uniform
  // words) holds the rows that fit its register budget, the rest stay scalar.
  static constexpr int RV_ROWS = !LIST || LIST2 ? N : list_rows(N, LS);
  static constexpr bool RUV = RV_ROWS > 0;
  static constexpr int WPE = LS >= 3 || LIST ? 4 : 1;
  // sets of each register stack slot that live in registers; the others sit
  // in the wave's LDS area (this keeps the eight-set census variant and the
  // seven- and eight-world four-set list variants within 128 VGPRs with
  // their relation rows in registers)
  static constexpr int SR = (RUV && LS >= 3) || list_four_sets(LIST, N, LS) ? S - 2 : S;
  // LDS words per lane: the LDS slots, then the register slots' LDS sets
  static constexpr int LDS_WORDS = (LDS_SLOTS * S + DS * (S - SR)) * N;
};

// Diagonal positions whose relation bit is shared by the whole block (mode K):
// a block can hold a reflexive frame only if all of them are set.
template <int N, int NV, int LS, int MODE>
__host__ __device__ constexpr uint64_t diag_uniform_mask() {
  uint64_t m = 0;
  for (int w = 0; w < N; ++w) {
    const int p = w * N + w;
    if (MODE == 0 && p >= Geo<N, NV, LS, MODE>::B) m |= 1ull << p;
  }
  return m;
}

template <int N, int NV, int LS, int MODE>
struct Ctx {
  using G = Geo<N, NV, LS, MODE>;
  uint32_t ru[N][N];                    // uniform relation words of the block (VGPRs if RUV)
  uint32_t pv[5];                       // in-word valuation patterns, kept in VGPRs
  uint32_t lm[G::LF > 0 ? G::LF : 1];   // per-lane frame-bit words
  uint32_t lv[G::LV > 0 ? G::LV : 1];   // per-lane valuation-bit words
  uint32_t ch[G::CHB > 0 ? G::CHB : 1]; // uniform valuation-chunk words
  uint32_t acc[G::S][N];
  uint32_t stk[G::DS][G::S][N];
  // this wave's LDS stack area, lane-minor: [LDS_SLOTS][S][N][64], then
  // [DS][S - SR][N][64] for the sets of the register slots held in LDS
  uint32_t* spill;
  int lane;
};

template <int N, int NV, int LS, int MODE>
__device__ __forceinline__ uint32_t rel(const Ctx<N, NV, LS, MODE>& c, int s, int w, int v) {
  using G = Geo<N, NV, LS, MODE>;
  const int p = w * N + v;
  const int ro = role<N, MODE, G::LF, LS>(p);
  if (ro == R_ONE) return ~0u;
  if (ro == R_LANE) return c.lm[role_idx<N, MODE>(p, 0)];
  if (ro == R_SET) return ((s >> role_idx<N, MODE>(p, G::LF)) & 1) ? ~0u : 0u;
  return c.ru[w][v];
}

template <int N, int NV, int LS, int MODE>
__device__ __forceinline__ uint32_t var_word(const Ctx<N, NV, LS, MODE>& c, int s, int i, int w) {
  using G = Geo<N, NV, LS, MODE>;
  const int b = i * N + w;
  if (b < 5) return c.pv[b];
  if (b < 5 + G::LV) return c.lv[b - 5];
  if (b < 5 + G::LV + G::SV) return ((s >> (b - 5 - G::LV)) & 1) ? ~0u : 0u;
  return c.ch[b - 5 - G::LV - G::SV];
}

template <int N, int NV, int LS, int MODE, int L>
__device__ __forceinline__ uint32_t leaf(const Ctx<N, NV, LS, MODE>& c, int s, int w) {
  if constexpr (L < 4) {
    return var_word(c, s, L, w);
  } else if constexpr (L < 8) {
    return ~var_word(c, s, L - 4, w);
  } else if constexpr (L == L_SUCC || L == L_DEAD) {
    // "has a successor": an OR over the row, seeded opaquely so it is
    // computed where used instead of being hoisted for every block
    uint32_t r;
    asm volatile("v_mov_b32 %0, 0" : "=v"(r));
#pragma unroll
    for (int v = 0; v < N; ++v) r |= rel(c, s, w, v);
    return L == L_SUCC ? r : ~r;
  } else if constexpr (L == L_TOP) {
    return ~0u;
  } else {
    return 0u;
  }
}

// Truth table of a 3-input bitwise function for v_bitop3: bit (a*4 + b*2 + c)
// of the immediate is f(a, b, c) for source operands (a, b, c).
template <typename F>
__host__ __device__ constexpr unsigned truth_table(F f) {
  unsigned t = 0;
  for (int i = 0; i < 8; ++i)
    if (f((i >> 2) & 1, (i >> 1) & 1, i & 1)) t |= 1u << i;
  return t;
}

// Binary connective of the accumulator with a variable literal, the
// literal's negation folded into the instruction: a loop-invariant ~x would
// otherwise be hoisted out of the interpreter loop and held in registers.
template <int OP, bool NEG>
__device__ __forceinline__ uint32_t bin_lit(uint32_t a, uint32_t x) {
  constexpr unsigned tt = truth_table([](int a, int x, int) {
    const int y = NEG ? !x : x;
    return OP == 0 ? (a & y) : OP == 1 ? (a | y) : (a == y);
  });
  return __builtin_amdgcn_bitop3_b32(a, x, x, tt);
}

// a == b bitwise as v_bitop3 (v_xnor_b32 issues at half rate on gfx950)
__device__ __forceinline__ uint32_t xnor3(uint32_t a, uint32_t b) {
  constexpr unsigned tt = truth_table([](int a, int b, int) { return a == b; });
  return __builtin_amdgcn_bitop3_b32(a, b, b, tt);
}

__device__ __forceinline__ uint32_t opaque_not(uint32_t x) {
  uint32_t r;
  asm volatile("v_not_b32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

#define KR_FOR_SW                    \
  _Pragma("unroll") for (int s = 0; s < Geo<N, NV, LS, MODE>::S; ++s) \
  _Pragma("unroll") for (int w = 0; w < N; ++w)

template <int N, int NV, int LS, int MODE, int L>
__device__ __forceinline__ void f_load(Ctx<N, NV, LS, MODE>& c) {
  if constexpr (L >= 4 && L < 8) {
    KR_FOR_SW c.acc[s][w] = opaque_not(var_word(c, s, L - 4, w));
  } else {
    KR_FOR_SW c.acc[s][w] = leaf<N, NV, LS, MODE, L>(c, s, w);
  }
}
template <int OP, int N, int NV, int LS, int MODE, int L>
__device__ __forceinline__ void f_bin_leaf(Ctx<N, NV, LS, MODE>& c) {
  if constexpr (L < 8) {
    KR_FOR_SW c.acc[s][w] = bin_lit<OP, (L >= 4)>(c.acc[s][w], var_word(c, s, L & 3, w));
  } else {
    KR_FOR_SW {
      const uint32_t y = leaf<N, NV, LS, MODE, L>(c, s, w);
      c.acc[s][w] = OP == 0 ? (c.acc[s][w] & y) : OP == 1 ? (c.acc[s][w] | y)
                                                          : xnor3(c.acc[s][w], y);
    }
  }
}
template <int N, int NV, int LS, int MODE, int L>
__device__ __forceinline__ void f_and(Ctx<N, NV, LS, MODE>& c) { f_bin_leaf<0, N, NV, LS, MODE, L>(c); }
template <int N, int NV, int LS, int MODE, int L>
__device__ __forceinline__ void f_or(Ctx<N, NV, LS, MODE>& c) { f_bin_leaf<1, N, NV, LS, MODE, L>(c); }
template <int N, int NV, int LS, int MODE, int L>
__device__ __forceinline__ void f_iff(Ctx<N, NV, LS, MODE>& c) { f_bin_leaf<2, N, NV, LS, MODE, L>(c); }
// Stack slots below DS live in registers (sets below SR; the others in the
// wave's LDS area); the next LDS_SLOTS live wholly in LDS (rare: only programs
// needing the extra slot touch it).
template <int N, int NV, int LS, int MODE>
__device__ __forceinline__ int lds_word(int d, int s, int w) {
  using G = Geo<N, NV, LS, MODE>;
  if (d >= G::DS) return ((d - G::DS) * G::S + s) * N + w;
  return G::LDS_SLOTS * G::S * N + (d * (G::S - G::SR) + (s - G::SR)) * N + w;
}
template <int N, int NV, int LS, int MODE>
__device__ __forceinline__ bool in_regs(int d, int s) {
  using G = Geo<N, NV, LS, MODE>;
  return d < G::DS && s < G::SR;
}
template <int N, int NV, int LS, int MODE, int D>
__device__ __forceinline__ void f_save(Ctx<N, NV, LS, MODE>& c) {
  using G = Geo<N, NV, LS, MODE>;
  if constexpr (D < G::DS + G::LDS_SLOTS) {
    KR_FOR_SW {
      if (in_regs<N, NV, LS, MODE>(D, s))
        c.stk[D < G::DS ? D : 0][s][w] = c.acc[s][w];
      else
        c.spill[lds_word<N, NV, LS, MODE>(D, s, w) * 64 + c.lane] = c.acc[s][w];
    }
  }
}
template <int N, int NV, int LS, int MODE, int D, int OP>
__device__ __forceinline__ void f_comb(Ctx<N, NV, LS, MODE>& c) {
  using G = Geo<N, NV, LS, MODE>;
  if constexpr (D < G::DS + G::LDS_SLOTS) {
    KR_FOR_SW {
      const uint32_t y = in_regs<N, NV, LS, MODE>(D, s)
                             ? c.stk[D < G::DS ? D : 0][s][w]
                             : c.spill[lds_word<N, NV, LS, MODE>(D, s, w) * 64 + c.lane];
      if constexpr (OP == 0) c.acc[s][w] &= y;
      else if constexpr (OP == 1) c.acc[s][w] |= y;
      else c.acc[s][w] = xnor3(c.acc[s][w], y);
    }
  }
}
constexpr unsigned kDiaTerm = truth_table([](int R, int t, int r) { return (R & t) | r; });
constexpr unsigned kBoxTerm = truth_table([](int R, int t, int r) { return r & (t | !R); });
constexpr unsigned kDiaTermN = truth_table([](int R, int t, int r) { return (R & !t) | r; });
constexpr unsigned kBoxTermN = truth_table([](int R, int t, int r) { return r & (!t | !R); });

// One (world w, successor v) term of Lemma 1: DIA accumulates R(w,v) & t_v
// into an OR, BOX accumulates ~R(w,v) | t_v into an AND.  Relation words that
// are compile-time constants (set bits, the reflexive diagonal) fold away.
template <bool DIA, int N, int NV, int LS, int MODE, bool NEG = false>
__device__ __forceinline__ uint32_t modal_term(const Ctx<N, NV, LS, MODE>& c, int s, int w, int v,
                                               uint32_t t, uint32_t r) {
  using G = Geo<N, NV, LS, MODE>;
  const int p = w * N + v;
  const int ro = role<N, MODE, G::LF, LS>(p);
  if (ro == R_ONE || (ro == R_SET && ((s >> role_idx<N, MODE>(p, G::LF)) & 1))) {
    constexpr unsigned tt = truth_table([](int t, int r, int) {
      const int u = NEG ? !t : t;
      return DIA ? (r | u) : (r & u);
    });
    return __builtin_amdgcn_bitop3_b32(t, r, r, tt);
  }
  if (ro == R_SET) return r;
  const uint32_t R = ro == R_LANE ? c.lm[role_idx<N, MODE>(p, 0)] : c.ru[w][v];
  return __builtin_amdgcn_bitop3_b32(
      R, t, r, DIA ? (NEG ? kDiaTermN : kDiaTerm) : (NEG ? kBoxTermN : kBoxTerm));
}

template <bool DIA, int N, int NV, int LS, int MODE>
__device__ __forceinline__ void f_modal(Ctx<N, NV, LS, MODE>& c) {
  // Every world's result reads every world's operand, so a set needs N
  // temporaries.  The empty asm ahead of each set orders the sets, and the
  // explicit moves retire the temporaries, so all sets share the same N
  // registers instead of the scheduler interleaving sets and holding S * N.
#pragma unroll
  for (int s = 0; s < Geo<N, NV, LS, MODE>::S; ++s) {
    uint32_t t[N];
#pragma unroll
    for (int w = 0; w < N; ++w) asm volatile("" : "+v"(c.acc[s][w]));
#pragma unroll
    for (int w = 0; w < N; ++w) {
      uint32_t r = DIA ? 0u : ~0u;
#pragma unroll
      for (int v = 0; v < N; ++v) r = modal_term<DIA>(c, s, w, v, c.acc[s][v], r);
      t[w] = r;
    }
#pragma unroll
    for (int w = 0; w < N; ++w) asm volatile("v_mov_b32 %0, %1" : "=v"(c.acc[s][w]) : "v"(t[w]));
  }
}

// Two modal operators in a row (one micro-op): the first writes temporaries,
// the second reads them and writes the accumulator directly, since the
// accumulator's old words are dead by then, so no retiring moves are needed.
template <bool DIA1, bool DIA2, int N, int NV, int LS, int MODE>
__device__ __forceinline__ void f_modal2(Ctx<N, NV, LS, MODE>& c) {
#pragma unroll
  for (int s = 0; s < Geo<N, NV, LS, MODE>::S; ++s) {
    uint32_t t[N];
#pragma unroll
    for (int w = 0; w < N; ++w) asm volatile("" : "+v"(c.acc[s][w]));
#pragma unroll
    for (int w = 0; w < N; ++w) {
      uint32_t r = DIA1 ? 0u : ~0u;
#pragma unroll
      for (int v = 0; v < N; ++v) r = modal_term<DIA1>(c, s, w, v, c.acc[s][v], r);
      t[w] = r;
    }
#pragma unroll
    for (int w = 0; w < N; ++w) asm volatile("" : "+v"(t[w]));
#pragma unroll
    for (int w = 0; w < N; ++w) {
      uint32_t r = DIA2 ? 0u : ~0u;
#pragma unroll
      for (int v = 0; v < N; ++v) r = modal_term<DIA2>(c, s, w, v, t[v], r);
      c.acc[s][w] = r;
    }
  }
}

// DIA/BOX applied directly to a literal: the literal's words are read in
// place instead of being loaded into the accumulator first.
template <bool DIA, int N, int NV, int LS, int MODE, int L>
__device__ __forceinline__ void f_modal_leaf(Ctx<N, NV, LS, MODE>& c) {
  static_assert(L < 8, "modal superinstructions take variable literals only");
  // Every operand of this handler is invariant inside a block, so without an
  // opaque seed the compiler would hoist all of these results out of the
  // interpreter loop and keep them live in registers.
  uint32_t seed;
  asm volatile("v_mov_b32 %0, %1" : "=v"(seed) : "i"(DIA ? 0 : -1));
#pragma unroll
  for (int s = 0; s < Geo<N, NV, LS, MODE>::S; ++s) {
#pragma unroll
    for (int w = 0; w < N; ++w) {
      uint32_t r = seed;
#pragma unroll
      for (int v = 0; v < N; ++v)
        r = modal_term<DIA, N, NV, LS, MODE, (L >= 4)>(c, s, w, v, var_word(c, s, L & 3, v), r);
      c.acc[s][w] = r;
    }
  }
}

#define KR_L10(BASE, FN)                                                               \
  case BASE + 0: FN(0); break; case BASE + 1: FN(1); break; case BASE + 2: FN(2); break; \
  case BASE + 3: FN(3); break; case BASE + 4: FN(4); break; case BASE + 5: FN(5); break; \
  case BASE + 6: FN(6); break; case BASE + 7: FN(7); break; case BASE + 8: FN(8); break; \
  case BASE + 9: FN(9); break;
#define KR_L8(BASE, FN)                                                                \
  case BASE + 0: FN(0); break; case BASE + 1: FN(1); break; case BASE + 2: FN(2); break; \
  case BASE + 3: FN(3); break; case BASE + 4: FN(4); break; case BASE + 5: FN(5); break; \
  case BASE + 6: FN(6); break; case BASE + 7: FN(7); break;
#define KR_D8(BASE, FN) \
  case BASE + 0: FN(0); break; case BASE + 1: FN(1); break; case BASE + 2: FN(2); break; \
  case BASE + 3: FN(3); break; case BASE + 4: FN(4); break; case BASE + 5: FN(5); break; \
  case BASE + 6: FN(6); break; case BASE + 7: FN(7); break;

// Interpret the wave's program (staged in LDS, 8-byte padded) on the current
// block.  Ops are consumed from a 64-bit shift register holding the next
// eight.  Only U_END and padding are zero bytes, so an all-zero register means
// the program ended or the register is exhausted, told apart by the number of
// 8-byte words left; that test is one scalar compare, so the end never goes
// through the dispatch tree.
template <int N, int NV, int LS, int MODE>
__device__ __forceinline__ void run(Ctx<N, NV, LS, MODE>& c, const uint32_t* prog, uint64_t first,
                                    uint32_t nwords) {
  uint64_t cur = first;
  uint32_t next = 1;
  for (;;) {
    if (cur == 0) {
      if (next >= nwords) return;
      cur = ((uint64_t)__builtin_amdgcn_readfirstlane(prog[2 * next + 1]) << 32) |
            __builtin_amdgcn_readfirstlane(prog[2 * next]);
      ++next;
      if ((cur & 0xffu) == 0) return;
    }
    const uint32_t op = (uint32_t)cur & 0xffu;
    cur >>= 8;
// Opcodes a program run by this variant cannot hold are unreachable: the
// host compiler rejects variables beyond nvars (= NV), and every launch
// path gives a variant only programs whose stack need fits its slots.
// Dropping those cases shortens the dispatch tree and the code.
#define KR_LEAF_OK(L) ((L) >= 8 || ((L) & 3) < NV)
#define KR_SLOT_OK(D) ((D) < Geo<N, NV, LS, MODE>::DS + Geo<N, NV, LS, MODE>::LDS_SLOTS)
#define KR_IF(OK, CALL) \
  if constexpr (OK) {   \
    CALL;               \
  } else {              \
    __builtin_unreachable(); \
  }
#define G_LOAD(L) KR_IF(KR_LEAF_OK(L), (f_load<N, NV, LS, MODE, L>(c)))
#define G_AND(L) KR_IF(KR_LEAF_OK(L), (f_and<N, NV, LS, MODE, L>(c)))
#define G_OR(L) KR_IF(KR_LEAF_OK(L), (f_or<N, NV, LS, MODE, L>(c)))
#define G_IFF(L) KR_IF(KR_LEAF_OK(L), (f_iff<N, NV, LS, MODE, L>(c)))
#define G_SAVE(D) KR_IF(KR_SLOT_OK(D), (f_save<N, NV, LS, MODE, D>(c)))
#define G_ANDS(D) KR_IF(KR_SLOT_OK(D), (f_comb<N, NV, LS, MODE, D, 0>(c)))
#define G_ORS(D) KR_IF(KR_SLOT_OK(D), (f_comb<N, NV, LS, MODE, D, 1>(c)))
#define G_IFFS(D) KR_IF(KR_SLOT_OK(D), (f_comb<N, NV, LS, MODE, D, 2>(c)))
#define G_DIAL(L) KR_IF(KR_LEAF_OK(L), (f_modal_leaf<true, N, NV, LS, MODE, L>(c)))
#define G_BOXL(L) KR_IF(KR_LEAF_OK(L), (f_modal_leaf<false, N, NV, LS, MODE, L>(c)))
    switch (op) {
      KR_L10(U_LOAD, G_LOAD)
      case U_LOAD + L_TOP: G_LOAD(L_TOP); break;
      case U_LOAD + L_BOT: G_LOAD(L_BOT); break;
      KR_L10(U_AND_L, G_AND)
      KR_L10(U_OR_L, G_OR)
      KR_L10(U_IFF_L, G_IFF)
      case U_BOX: f_modal<false, N, NV, LS, MODE>(c); break;
      case U_DIA: f_modal<true, N, NV, LS, MODE>(c); break;
      KR_D8(U_SAVE, G_SAVE)
      KR_D8(U_AND_S, G_ANDS)
      KR_D8(U_OR_S, G_ORS)
      KR_D8(U_IFF_S, G_IFFS)
      KR_L8(U_DIA_L, G_DIAL)
      KR_L8(U_BOX_L, G_BOXL)
      case U_MM + 0: f_modal2<false, false, N, NV, LS, MODE>(c); break;
      case U_MM + 1: f_modal2<false, true, N, NV, LS, MODE>(c); break;
      case U_MM + 2: f_modal2<true, false, N, NV, LS, MODE>(c); break;
      case U_MM + 3: f_modal2<true, true, N, NV, LS, MODE>(c); break;
      default: __builtin_unreachable();
    }
    // Pinning the accumulator at the end of every handler lets the register
    // allocator give it one home across the loop; without this it carries a
    // few words in a second set of registers, copied back on every micro-op.
#pragma unroll
    for (int s = 0; s < Geo<N, NV, LS, MODE>::S; ++s)
#pragma unroll
      for (int w = 0; w < N; ++w) asm volatile("" : "+v"(c.acc[s][w]));
#undef KR_IF
#undef KR_LEAF_OK
#undef KR_SLOT_OK
#undef G_LOAD
#undef G_AND
#undef G_OR
#undef G_IFF
#undef G_SAVE
#undef G_ANDS
#undef G_ORS
#undef G_IFFS
#undef G_DIAL
#undef G_BOXL
  }
}

// Candidate key of the least failing model among the lanes' bits for one
// (set, chunk) pass: the lowest failing lane holds the least frame and then
// the least valuation, and the lowest failing bit its least in-word bits.
template <int N, int NV, int LS, int MODE>
__device__ __forceinline__ uint64_t candidate(const Ctx<N, NV, LS, MODE>& c, int s, uint32_t fail,
                                              uint64_t bal, uint64_t blk, uint32_t chunk,
                                              int lane) {
  using G = Geo<N, NV, LS, MODE>;
  const int fl = __builtin_ctzll(bal);
  const uint32_t j = __builtin_ctz(fail | 0x80000000u);
  // the least world where the program is false (world 0 for an all-fail
  // program, whose accumulator is zero)
  uint32_t world = 0;
#pragma unroll
  for (int w = N - 1; w >= 0; --w)
    if (!((c.acc[s][w] >> j) & 1u)) world = w;
  // list mode: the key's frame field is the list position, and the set is a
  // valuation field
  const uint64_t pos = G::LIST2  ? (blk << G::B) | (uint64_t)(lane >> G::LV)
                       : G::LIST ? blk
                                 : (blk << G::B) | ((uint64_t)s << G::LF) | (uint64_t)(lane >> G::LV);
  const uint64_t frame = MODE == 1 ? refl_frame(pos, N) : pos;
  const uint64_t val = ((uint64_t)chunk << (5 + G::LV + G::SV)) |
                       (G::LIST ? (uint64_t)s << (5 + G::LV) : 0ull) |
                       ((uint64_t)(lane & ((1 << G::LV) - 1)) << 5) | j;
  const uint64_t lk = (frame << (G::V + 4)) | (val << 4) | world;
  return readlane64(lk, fl);
}

// Words of one staged program (the micro-ops, 8-byte padded, and slack).
constexpr int kProgWords = kMaxMicro / 4 + 4;

// Stage the programs of a list work item's formula group (formulas f0 ..
// f0 + ng - 1 of the launch order) side by side in the wave's LDS area.  A
// formula whose known key precedes the item's first position p0, or whose
// program is TOP (no countermodel), takes no part; live gets bit j for the
// others, bot bit j for a BOT program (false everywhere, not interpreted).
template <int V>
__device__ __forceinline__ void stage_group(const FastArgs& a, uint32_t (*progs)[kProgWords],
                                            uint32_t* pws, uint32_t f0, uint32_t ng,
                                            uint64_t p0, int lane, uint32_t& live,
                                            uint32_t& bot) {
  live = 0;
  bot = 0;
  for (uint32_t j = 0; j < ng; ++j) {
    const uint32_t f = a.order[f0 + j];
    uint64_t known = __hip_atomic_load(a.out_key + (uint64_t)f * a.out_stride, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
    known = readlane64(known, 0);
    if (known != ~0ull && (known >> (V + 4)) < p0) continue;
    const uint32_t q0 = a.uoff[f] >> 2, pw = (a.uoff[f + 1] >> 2) - q0;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.ucode) + q0;
    for (uint32_t i = lane; i < pw; i += 64) progs[j][i] = src[i];
    const uint64_t first = ((uint64_t)__builtin_amdgcn_readfirstlane(src[1]) << 32) |
                           __builtin_amdgcn_readfirstlane(src[0]);
    if (first == (uint64_t)(U_LOAD + L_TOP)) continue;
    if (first == (uint64_t)(U_LOAD + L_BOT)) bot |= 1u << j;
    if (lane == 0) pws[j] = pw;
    live |= 1u << j;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One work item of mode 2: a range of one-frame list blocks for a group of up
// to kListGroupMax formulas, first keys only.  Each block's frame rows are
// read once (scalar loads) and decoded once; every formula of the group
// without a key then runs its valuation chunks in increasing order, and the
// first chunk with a failure holds the frame's least key for that formula
// (chunk bits are the highest valuation bits): the key goes out at once and
// the formula leaves the group.
template <int N, int NV, int LS>
__device__ __forceinline__ void list_item(const FastArgs& a, Ctx<N, NV, LS, 2>& c,
                                          uint32_t (*progs)[kProgWords], uint32_t* pws,
                                          uint64_t item, int lane) {
  using G = Geo<N, NV, LS, 2>;
  static_assert(G::B == 0, "a list block is one list position");
  const uint64_t blk_end = a.blk_begin + a.nblk;
  const uint32_t f0 = (uint32_t)(item / a.items_per_formula) * a.group;
  const uint32_t ng = a.nformulas - f0 < a.group ? a.nformulas - f0 : a.group;
  const uint64_t b0 = a.blk_begin + (item % a.items_per_formula) * a.blocks_per_item;
  const uint64_t b1 = b0 + a.blocks_per_item < blk_end ? b0 + a.blocks_per_item : blk_end;
  uint32_t live = 0, bot = 0;
  const uint64_t p0 = b0 > a.pos_begin ? b0 : a.pos_begin;
  stage_group<G::V>(a, progs, pws, f0, ng, p0, lane, live, bot);

  for (uint64_t blk = b0; blk < b1 && live; ++blk) {
    // the frame's successor rows, wave-uniform: the list is read-only for the
    // kernel's lifetime, so reading it through the constant address space
    // gives scalar loads straight into SGPRs
    const __attribute__((address_space(4))) uint32_t* rows =
        (const __attribute__((address_space(4))) uint32_t*)(uintptr_t)(a.list_succ + blk * N);
    uint64_t base = 0;
#pragma unroll
    for (int w = 0; w < N; ++w) base |= (uint64_t)rows[w] << (w * N);
    // the first RV_ROWS rows in vector registers, one signed bit-field
    // extract per word (opaque, so the words stay vector values); the others
    // stay scalar
    uint32_t vbase[2] = {0u, 0u};
    if constexpr (G::RUV) {
      asm volatile("v_mov_b32 %0, %1" : "=v"(vbase[0]) : "s"((uint32_t)base));
      if constexpr (N * G::RV_ROWS > 32)
        asm volatile("v_mov_b32 %0, %1" : "=v"(vbase[1]) : "s"((uint32_t)(base >> 32)));
    }
#pragma unroll
    for (int w = 0; w < N; ++w)
#pragma unroll
      for (int v = 0; v < N; ++v) {
        const int p = w * N + v;
        if (w < G::RV_ROWS) {
          uint32_t r;
          asm volatile("v_bfe_i32 %0, %1, %2, 1" : "=v"(r) : "v"(vbase[p >> 5]), "i"(p & 31));
          c.ru[w][v] = r;
        } else if (N * N <= 32) {
          c.ru[w][v] = (uint32_t)__builtin_amdgcn_sbfe((int)(uint32_t)base, p, 1);
        } else {
          c.ru[w][v] = 0u - (uint32_t)((base >> p) & 1u);
        }
      }
    for (uint32_t j = 0; j < ng; ++j) {
      if (!((live >> j) & 1u)) continue;
      const uint32_t* prog = progs[j];
      for (uint32_t chunk = 0; chunk < (1u << G::CHB); ++chunk) {
#pragma unroll
        for (int i = 0; i < G::CHB; ++i)
          c.ch[i] = (uint32_t)__builtin_amdgcn_readfirstlane((int)(0u - ((chunk >> i) & 1u)));
        if ((bot >> j) & 1u) {
#pragma unroll
          for (int s = 0; s < G::S; ++s)
#pragma unroll
            for (int w = 0; w < N; ++w) c.acc[s][w] = 0u;
        } else {
          const uint64_t first = ((uint64_t)__builtin_amdgcn_readfirstlane(prog[1]) << 32) |
                                 __builtin_amdgcn_readfirstlane(prog[0]);
          run<N, NV, LS, 2>(c, prog, first, (uint32_t)__builtin_amdgcn_readfirstlane(pws[j]) >> 1);
        }
        // any failure on this lane: one AND over every set's words
        uint32_t holds = ~0u;
#pragma unroll
        for (int s = 0; s < G::S; ++s)
#pragma unroll
          for (int w = 0; w < N; ++w) holds &= c.acc[s][w];
        if (!__ballot(holds != ~0u)) continue;
        // the least key lies in the first failing set (sets are valuation
        // bits above the lane bits)
        uint64_t best = ~0ull;
        bool found = false;
#pragma unroll
        for (int s = 0; s < G::S; ++s) {
          if (!found) {
            uint32_t all = ~0u;
#pragma unroll
            for (int w = 0; w < N; ++w) all &= c.acc[s][w];
            const uint32_t fail = ~all;
            const uint64_t bal = __ballot(fail != 0);
            if (bal) {
              best = candidate(c, s, fail, bal, blk, chunk, lane);
              found = true;
            }
          }
        }
        if (lane == 0)
          atomicMin(a.out_key + (uint64_t)a.order[f0 + j] * a.out_stride,
                    (unsigned long long)best);
        live = (uint32_t)__builtin_amdgcn_readfirstlane((int)(live & ~(1u << j)));
        break;
      }
    }
  }
}

// One work item of mode 3: a range of two-frame blocks for a group of up to
// kListGroupMax formulas (consecutive in the launch order), first keys only.
// The group's programs are staged side by side in the wave's LDS area; each
// block's two frames are loaded and decoded once, then every formula of the
// group without a key is interpreted on them.  A formula's first failing
// block holds its least key in the range (blocks run in increasing position
// order); the key goes out at once and the formula leaves the group.
template <int N, int NV, int LS>
__device__ __forceinline__ void list2_item(const FastArgs& a, Ctx<N, NV, LS, 3>& c,
                                           uint32_t (*progs)[kProgWords], uint32_t* pws,
                                           uint64_t item, int lane, uint64_t rag_lo,
                                           uint64_t rag_hi) {
  using G = Geo<N, NV, LS, 3>;
  static_assert(G::CHB == 0, "a two-frame block holds all valuations of its frames");
  const uint32_t lane_pos = (uint32_t)(lane >> G::LV);
  const uint64_t blk_end = a.blk_begin + a.nblk;
  const uint32_t f0 = (uint32_t)(item / a.items_per_formula) * a.group;
  const uint32_t ng = a.nformulas - f0 < a.group ? a.nformulas - f0 : a.group;
  const uint64_t b0 = a.blk_begin + (item % a.items_per_formula) * a.blocks_per_item;
  const uint64_t b1 = b0 + a.blocks_per_item < blk_end ? b0 + a.blocks_per_item : blk_end;
  const uint64_t p0 = (b0 << G::B) > a.pos_begin ? (b0 << G::B) : a.pos_begin;

  uint32_t live = 0, bot = 0;
  stage_group<G::V>(a, progs, pws, f0, ng, p0, lane, live, bot);

  for (uint64_t blk = b0; blk < b1 && live; ++blk) {
    // each half-wave's frame (position blk << B | lane_pos; a position past
    // the list end, in a ragged last block, loads the last frame and is masked
    // out of the failure test) as per-lane relation words, one signed
    // bit-field extract per word from the lane's successor rows
    const uint64_t pbase = blk << G::B;
    {
      uint64_t fp = pbase | lane_pos;
      if (fp >= a.pos_end) fp = a.pos_end - 1;
      const uint32_t* r = a.list_succ + fp * N;
      uint32_t row[N];
#pragma unroll
      for (int w = 0; w < N; ++w) row[w] = r[w];
#pragma unroll
      for (int w = 0; w < N; ++w)
#pragma unroll
        for (int v = 0; v < N; ++v) {
          uint32_t x;
          asm volatile("v_bfe_i32 %0, %1, %2, 1" : "=v"(x) : "v"(row[w]), "i"(v));
          c.ru[w][v] = x;
        }
    }
    bool in_range = true;
    if (blk == rag_lo || blk == rag_hi) {
      const uint64_t pos = pbase | lane_pos;
      in_range = pos >= a.pos_begin && pos < a.pos_end;
    }
    for (uint32_t j = 0; j < ng; ++j) {
      if (!((live >> j) & 1u)) continue;
      if ((bot >> j) & 1u) {
        // BOT is false everywhere: a zero accumulator, no interpretation
#pragma unroll
        for (int s = 0; s < G::S; ++s)
#pragma unroll
          for (int w = 0; w < N; ++w) c.acc[s][w] = 0u;
      } else {
        const uint32_t* prog = progs[j];
        const uint64_t first = ((uint64_t)__builtin_amdgcn_readfirstlane(prog[1]) << 32) |
                               __builtin_amdgcn_readfirstlane(prog[0]);
        run<N, NV, LS, 3>(c, prog, first, (uint32_t)__builtin_amdgcn_readfirstlane(pws[j]) >> 1);
      }
      // failing (valuation) bits of set s on this lane
      auto fail_of = [&](int s) {
        uint32_t all = ~0u;
#pragma unroll
        for (int w = 0; w < N; ++w) all &= c.acc[s][w];
        return in_range ? ~all : 0u;
      };
      // any failure on this lane: one AND over every set's words
      uint32_t holds = ~0u;
#pragma unroll
      for (int s = 0; s < G::S; ++s)
#pragma unroll
        for (int w = 0; w < N; ++w) holds &= c.acc[s][w];
      const uint32_t anyfail = in_range ? ~holds : 0u;
      if (!__ballot(anyfail != 0)) continue;
      // the first half-wave's frame precedes every valuation of the second:
      // the sets are searched on its lanes first, then on the whole wave
      uint64_t best = ~0ull;
      bool found = false;
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const uint64_t lanes = half == 0 ? 0xFFFFFFFFull : ~0ull;
#pragma unroll
        for (int s = 0; s < G::S; ++s) {
          if (!found) {
            const uint32_t fail = fail_of(s);
            const uint64_t bal = __ballot(fail != 0) & lanes;
            if (bal) {
              const uint64_t k = candidate(c, s, fail, bal, blk, 0u, lane);
              best = k < best ? k : best;
              found = true;
            }
          }
        }
      }
      if (lane == 0)
        atomicMin(a.out_key + (uint64_t)a.order[f0 + j] * a.out_stride, (unsigned long long)best);
      live = (uint32_t)__builtin_amdgcn_readfirstlane((int)(live & ~(1u << j)));
    }
  }
}

template <int N, int NV, int LS, int MODE, bool FUSED>
// The eight-set and list variants are sized for four waves per SIMD.
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(Geo<N, NV, LS, MODE>::WPE)))
void census_fast(FastArgs a) {
  using G = Geo<N, NV, LS, MODE>;
  static_assert(G::V >= 5, "fast kernel needs n * nvars >= 5");
  static_assert(!G::LIST || (G::V >= 5 + G::LV + LS && !FUSED),
                "list mode needs the lane and set bits to be valuation bits");
  // staged programs: one per wave, a group of them in mode 3
  __shared__ uint32_t sprog[4][G::LIST ? kListGroupMax : 1][kProgWords];
  __shared__ uint32_t spw[4][G::LIST ? kListGroupMax : 1];
  __shared__ uint32_t sspill[4][G::LDS_WORDS > 0 ? G::LDS_WORDS * 64 : 1];
  // fused mode: per-lane failure counts of the classes T, S4, S5, private to
  // the lane (only blocks that can hold a reflexive frame touch them, so they
  // need not occupy registers through the interpreter)
  __shared__ uint32_t scls[4][FUSED ? 3 : 1][64];
  const int lane = threadIdx.x & 63;
  uint32_t* prog = sprog[threadIdx.x >> 6][0];
  constexpr int NC = FUSED ? 4 : 1;
  const uint64_t blk_end = a.blk_begin + a.nblk;

  Ctx<N, NV, LS, MODE> c;
  c.spill = sspill[threadIdx.x >> 6];
  c.lane = lane;
  // Patterns live in vector registers on purpose: a modal term combines a
  // scalar relation word with a pattern, and an instruction takes at most one
  // scalar operand.
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    uint32_t v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(pattern(b)));
    c.pv[b] = v;
  }
#pragma unroll
  for (int i = 0; i < G::LF; ++i) c.lm[i] = 0u - ((lane >> (G::LV + i)) & 1u);
#pragma unroll
  for (int i = 0; i < G::LV; ++i) c.lv[i] = 0u - ((lane >> i) & 1u);
  const uint32_t lane_pos = (uint32_t)(lane >> G::LV);
  // only the first and the last block can hold positions outside the range
  constexpr uint64_t kBlockMask = (1ull << G::B) - 1;
  const uint64_t rag_lo = (a.pos_begin & kBlockMask) ? (a.pos_begin >> G::B) : ~0ull;
  const uint64_t rag_hi = (a.pos_end & kBlockMask) ? ((a.pos_end - 1) >> G::B) : ~0ull;

  for (;;) {
    uint64_t item = 0;
    if (lane == 0) item = atomicAdd(a.queue, 1ull);
    item = readlane64(item, 0);
    if (item >= a.total_items) break;
    if constexpr (G::LIST2) {
      list2_item<N, NV, LS>(a, c, sprog[threadIdx.x >> 6], spw[threadIdx.x >> 6], item, lane,
                            rag_lo, rag_hi);
      continue;
    } else if constexpr (G::LIST) {
      list_item<N, NV, LS>(a, c, sprog[threadIdx.x >> 6], spw[threadIdx.x >> 6], item, lane);
      continue;
    }
    // (list-mode items never reach this point)
    const uint32_t f = a.order[item / a.items_per_formula];
    const uint64_t b0 = a.blk_begin + (item % a.items_per_formula) * a.blocks_per_item;
    const uint64_t b1 = b0 + a.blocks_per_item < blk_end ? b0 + a.blocks_per_item : blk_end;
    unsigned long long* key_out = a.out_key + (uint64_t)f * a.out_stride;

    if (a.decide) {
      const uint64_t p0 = (b0 << G::B) > a.pos_begin ? (b0 << G::B) : a.pos_begin;
      const uint64_t first_frame = MODE == 1 ? refl_frame(p0, N) : p0;
      uint64_t known = __hip_atomic_load(key_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      known = readlane64(known, 0);
      if (known != ~0ull && (known >> (G::V + 4)) < first_frame) continue;
    }

    const uint32_t p0 = a.uoff[f] >> 2, pw = (a.uoff[f + 1] >> 2) - p0;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.ucode) + p0;
    for (uint32_t i = lane; i < pw; i += 64) prog[i] = src[i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint64_t first = ((uint64_t)__builtin_amdgcn_readfirstlane(prog[1]) << 32) |
                           __builtin_amdgcn_readfirstlane(prog[0]);
    // TOP holds everywhere: no countermodel, nothing to scan.  BOT fails at
    // world 0 of every model: every block is all-fail without interpretation.
    if (first == (uint64_t)(U_LOAD + L_TOP)) continue;
    // BOT is false everywhere: no interpretation, a zero accumulator
    const bool all_fail = first == (uint64_t)(U_LOAD + L_BOT);
    if (all_fail) {
#pragma unroll
      for (int s = 0; s < G::S; ++s)
#pragma unroll
        for (int w = 0; w < N; ++w) c.acc[s][w] = 0u;
    }

    uint32_t cnt0 = 0;
    uint32_t* ccls = &scls[threadIdx.x >> 6][0][lane];  // class k at ccls[(k - 1) * 64]
    if constexpr (FUSED) {
#pragma unroll
      for (int k = 1; k < NC; ++k) ccls[(k - 1) * 64] = 0;
    }
    uint64_t key[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) key[k] = ~0ull;
    bool done = false;

    for (uint64_t blk = b0; blk < b1 && !done; ++blk) {
      const uint64_t pbase = blk << G::B;
      const uint64_t base = MODE == 0 ? pbase : refl_frame(pbase, N);
      // the relation bits in vector registers, expanded there by one signed
      // bit-field extract per word (opaque, so the words stay vector values)
      uint32_t vbase[2] = {0u, 0u};
      if constexpr (G::RUV) {
        asm volatile("v_mov_b32 %0, %1" : "=v"(vbase[0]) : "s"((uint32_t)base));
        if constexpr (N * G::RV_ROWS > 32)
          asm volatile("v_mov_b32 %0, %1" : "=v"(vbase[1]) : "s"((uint32_t)(base >> 32)));
      }
#pragma unroll
      for (int w = 0; w < N; ++w)
#pragma unroll
        for (int v = 0; v < N; ++v) {
          const int p = w * N + v;
          if (role<N, MODE, G::LF, LS>(p) != R_UNIFORM) continue;
          if (w < G::RV_ROWS) {
            uint32_t r;
            asm volatile("v_bfe_i32 %0, %1, %2, 1" : "=v"(r) : "v"(vbase[p >> 5]), "i"(p & 31));
            c.ru[w][v] = r;
          } else if (N * N <= 32) {  // one scalar signed bit-field extract per word
            c.ru[w][v] = (uint32_t)__builtin_amdgcn_sbfe((int)(uint32_t)base, p, 1);
          } else {
            c.ru[w][v] = 0u - (uint32_t)((base >> p) & 1u);
          }
        }
      // valid (lane, set) pairs: positions inside [pos_begin, pos_end)
      const bool ragged = blk == rag_lo || blk == rag_hi;
      // class levels of the block's frames; consumed only after evaluation,
      // so the scalar load overlaps the interpreter
      uint32_t lvl_raw = 0;
      constexpr uint64_t kDiag = diag_uniform_mask<N, NV, LS, MODE>();
      if (FUSED && (base & kDiag) == kDiag)
        lvl_raw = a.levels[pbase >> 4];
      uint64_t best[NC];
#pragma unroll
      for (int k = 0; k < NC; ++k) best[k] = ~0ull;
      // frame validity bits of the block's 2^B frames (validity maps only)
      constexpr bool kMaps = !FUSED && !G::LIST && G::CHB == 0 && G::B <= 5;
      uint32_t vbits = 0;

      for (uint32_t chunk = 0; chunk < (1u << G::CHB); ++chunk) {
#pragma unroll
        for (int i = 0; i < G::CHB; ++i)
          c.ch[i] = (uint32_t)__builtin_amdgcn_readfirstlane((int)(0u - ((chunk >> i) & 1u)));
        if (!all_fail) run<N, NV, LS, MODE>(c, prog, first, pw >> 1);
        const uint32_t lvl_word = FUSED ? __builtin_amdgcn_readfirstlane(
                                              lvl_raw >> ((uint32_t)(pbase & 15) * 2))
                                        : 0u;
        const bool classy = FUSED && (lvl_word & (G::B >= 4 ? 0xFFFFFFFFu
                                                  : ((1u << (2 << G::B)) - 1u))) != 0;
        // failing (valuation) bits of set s on this lane
        auto fail_of = [&](int s) {
          uint32_t all = ~0u;
#pragma unroll
          for (int w = 0; w < N; ++w) all &= c.acc[s][w];
          uint32_t fail = ~all;  // an all-fail program's accumulator is zero
          if (ragged) {
            const uint64_t pos = pbase | ((uint64_t)s << G::LF) | lane_pos;
            if (pos < a.pos_begin || pos >= a.pos_end) fail = 0;
          }
          return fail;
        };
        uint32_t anyfail = 0;
        // the common block (no range edge, no frame of a narrower class, no
        // validity map) tests its uniform conditions once, not per set
        const bool plain = !ragged && !classy && !(kMaps && a.valid_bits);
        if (plain && key[0] != ~0ull) {
          // the item's least key is known: failures are only counted
#pragma unroll
          for (int s = 0; s < G::S; ++s) {
            uint32_t all = ~0u;
#pragma unroll
            for (int w = 0; w < N; ++w) all &= c.acc[s][w];
            cnt0 += __builtin_popcount(~all);
          }
        } else if (plain) {
#pragma unroll
          for (int s = 0; s < G::S; ++s) {
            uint32_t all = ~0u;
#pragma unroll
            for (int w = 0; w < N; ++w) all &= c.acc[s][w];
            cnt0 += __builtin_popcount(~all);
            anyfail |= ~all;
          }
        } else {
#pragma unroll
          for (int s = 0; s < G::S; ++s) {
            const uint32_t fail = fail_of(s);
            cnt0 += __builtin_popcount(fail);
            if constexpr (kMaps) {
              if (a.valid_bits) {
                // a frame's valuations fill 2^LV consecutive lanes: it is valid
                // iff none of them holds a failing bit
                const uint64_t bal = __ballot(fail != 0);
                constexpr uint64_t kGroup = G::LV == 6 ? ~0ull : (1ull << (1 << G::LV)) - 1;
                uint32_t inv = 0;
#pragma unroll
                for (int g = 0; g < (1 << G::LF); ++g)
                  if ((bal >> (g << G::LV)) & kGroup) inv |= 1u << g;
                vbits |= (~inv & ((1u << (1 << G::LF)) - 1u)) << (s << G::LF);
              }
            }
            anyfail |= fail;
            if constexpr (FUSED) {
              if (classy) {
                const uint32_t lvl = (lvl_word >> (2 * ((s << G::LF) | lane_pos))) & 3u;
#pragma unroll
                for (int k = 1; k < NC; ++k) {
                  const uint32_t fk = lvl >= (uint32_t)k ? fail : 0u;
                  ccls[(k - 1) * 64] += __builtin_popcount(fk);
                  if (key[k] == ~0ull) {
                    const uint64_t bal = __ballot(fk != 0);
                    if (bal) {
                      const uint64_t kk = candidate(c, s, fk, bal, blk, chunk, lane);
                      best[k] = kk < best[k] ? kk : best[k];
                    }
                  }
                }
              }
            }
          }
        }
        // one ballot per block while no key is known; then the least key lies in
        // the first failing set (sets follow frame positions)
        if (key[0] == ~0ull && __ballot(anyfail != 0)) {
          bool found = false;
#pragma unroll
          for (int s = 0; s < G::S; ++s) {
            if (!found) {
              const uint32_t fail = fail_of(s);
              const uint64_t bal = __ballot(fail != 0);
              if (bal) {
                const uint64_t k = candidate(c, s, fail, bal, blk, chunk, lane);
                best[0] = k < best[0] ? k : best[0];
                found = true;
              }
            }
          }
        }
      }
#pragma unroll
      for (int k = 0; k < NC; ++k)
        if (key[k] == ~0ull) key[k] = best[k];
      if constexpr (kMaps) {
        if (a.valid_bits && vbits && lane == 0)
          atomicOr(a.valid_bits + (uint64_t)f * a.valid_words + (pbase >> 5),
                   vbits << (uint32_t)(pbase & 31));
      }
      if (a.decide && key[0] != ~0ull) done = true;
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      uint32_t ck = k == 0 ? cnt0 : ccls[(k > 0 ? k - 1 : 0) * 64];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) ck += __shfl_xor(ck, o);
      if (lane == 0) {
        if (key[k] != ~0ull) atomicMin(key_out + k * a.class_stride, (unsigned long long)key[k]);
        if (ck && a.out_cnt)
          atomicAdd(a.out_cnt + (uint64_t)f * a.out_stride + k * a.class_stride,
                    (unsigned long long)ck);
      }
    }
  }
}

// Class levels (0 K, 1 T, 2 S4, 3 S5), 2 bits per frame, 16 frames per word.
__global__ void build_levels(int n, uint64_t nwords, uint32_t* levels) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nwords) return;
  const uint32_t full = (1u << n) - 1u;
  uint32_t word = 0;
  for (int k = 0; k < 16; ++k) {
    const uint64_t f = i * 16 + k;
    if (f >> (n * n)) break;
    uint32_t succ[8];
    for (int w = 0; w < n; ++w) succ[w] = (uint32_t)(f >> (w * n)) & full;
    int lvl = 3;
    for (int w = 0; w < n && lvl; ++w)
      if (!((succ[w] >> w) & 1u)) lvl = 0;
    for (int w = 0; w < n && lvl > 1; ++w)
      for (int v = 0; v < n; ++v)
        if (((succ[w] >> v) & 1u) && (succ[v] & ~succ[w])) lvl = 1;
    for (int w = 0; w < n && lvl > 2; ++w)
      for (int v = 0; v < n; ++v)
        if (((succ[w] >> v) & 1u) != ((succ[v] >> w) & 1u)) lvl = 2;
    word |= (uint32_t)lvl << (2 * k);
  }
  levels[i] = word;
}

template <int N, int NV, int LS, int MODE, bool FUSED>
hipError_t launch_t(const FastArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((census_fast<N, NV, LS, MODE, FUSED>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Resident blocks per CU, queried once per variant (the query costs about a
// millisecond of host time, which per-formula launch loops would pay each time).
template <int N, int NV, int LS, int MODE, bool FUSED>
int occ_t() {
  static std::atomic<int> cached{0};
  int b = cached.load(std::memory_order_relaxed);
  if (b > 0) return b;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, census_fast<N, NV, LS, MODE, FUSED>, 256,
                                                   0) != hipSuccess ||
      b <= 0)
    return 1;
  cached.store(b, std::memory_order_relaxed);
  return b;
}

struct Entry {
  int n, nvars, ls, mode, fused;
  hipError_t (*launch)(const FastArgs&, int, hipStream_t);
  int (*occ)();
  int slots;  // stack slots: registers plus LDS
};

#define KR_E(N, NV, LS, MODE, F)                                                    \
  {N, NV, LS, MODE, F, &launch_t<N, NV, LS, MODE, F>, &occ_t<N, NV, LS, MODE, F>, \
   Geo<N, NV, LS, MODE>::DS + Geo<N, NV, LS, MODE>::LDS_SLOTS}
const Entry kTable[] = {
    KR_E(5, 2, 0, 0, false), KR_E(5, 2, 1, 0, false), KR_E(5, 2, 2, 0, false),
    KR_E(5, 2, 0, 0, true),  KR_E(5, 2, 1, 0, true),  KR_E(5, 2, 2, 0, true),
    KR_E(5, 2, 3, 0, false), KR_E(5, 2, 3, 0, true),  KR_E(5, 2, 3, 1, false),
    KR_E(5, 2, 0, 1, false), KR_E(5, 2, 1, 1, false), KR_E(5, 2, 2, 1, false),
    KR_E(5, 3, 0, 0, false), KR_E(5, 3, 1, 0, false), KR_E(5, 3, 1, 1, false),
    KR_E(5, 3, 1, 0, true),
    KR_E(4, 3, 0, 0, false), KR_E(4, 3, 1, 0, false), KR_E(4, 3, 1, 1, false),
    KR_E(4, 3, 1, 0, true),
    KR_E(4, 2, 1, 0, false), KR_E(4, 2, 1, 1, false), KR_E(4, 2, 1, 0, true),
    KR_E(6, 2, 0, 0, false), KR_E(6, 2, 1, 0, false), KR_E(6, 2, 1, 1, false),
    // frame lists (split search)
    KR_E(6, 2, 0, 2, false), KR_E(6, 2, 1, 2, false),
    KR_E(7, 2, 0, 2, false), KR_E(7, 2, 1, 2, false), KR_E(7, 2, 2, 2, false),
    KR_E(8, 2, 0, 2, false), KR_E(8, 2, 1, 2, false), KR_E(8, 2, 2, 2, false),
    // two frames per block
    KR_E(6, 2, 2, 3, false),
};

const Entry* find(int n, int nvars, int ls, int mode, bool fused) {
  for (const Entry& e : kTable)
    if (e.n == n && e.nvars == nvars && e.ls == ls && e.mode == mode && e.fused == (int)fused)
      return &e;
  return nullptr;
}

}  // namespace

bool fast_available(int n, int nvars, int ls, int mode, bool fused) {
  return find(n, nvars, ls, mode, fused) != nullptr;
}

int fast_block_log2(int n, int nvars, int ls, int mode) {
  if (mode == 2) return 0;
  if (mode == 3) return 1;
  const int V = n * nvars;
  const int lv = V >= 11 ? 6 : (V > 5 ? V - 5 : 0);
  return 6 - lv + ls;
}

hipError_t launch_fast(const FastArgs& a, int n, int nvars, int ls, int mode, bool fused, int grid,
                       hipStream_t s) {
  const Entry* e = find(n, nvars, ls, mode, fused);
  if (!e) return hipErrorInvalidValue;
  return e->launch(a, grid, s);
}

int fast_stack_slots(int n, int nvars, int ls, int mode, bool fused) {
  const Entry* e = find(n, nvars, ls, mode, fused);
  return e ? e->slots : 0;
}

int fast_blocks_per_cu(int n, int nvars, int ls, int mode, bool fused) {
  const Entry* e = find(n, nvars, ls, mode, fused);
  return e ? e->occ() : 1;
}

hipError_t launch_levels(int n, uint32_t* levels, hipStream_t s) {
  const uint64_t nwords = ((1ull << (n * n)) + 15) / 16;
  hipLaunchKernelGGL(build_levels, dim3((uint32_t)((nwords + 255) / 256)), dim3(256), 0, s, n,
                     nwords, levels);
  return hipGetLastError();
}

uint64_t refl_frame_host(uint64_t j, int n) { return refl_frame(j, n); }

}  // namespace kripke
