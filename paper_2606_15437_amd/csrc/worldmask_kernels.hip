// Split search on large frames: world-set bitmasks per lane.
//
// The bit-sliced kernels hold the relation as n*n words, which does not scale
// past ten worlds.  Here every lane evaluates one (frame, valuation) pair of a
// caller's frame list with truth sets as n-bit masks (bit w = the subformula
// holds at world w), the representation of Lemma 1: BOX t holds at w iff
// succ(w) is contained in t, DIA t iff succ(w) meets t.  A frame costs n
// registers of successor masks; formulas are the same compiled micro-op
// programs as everywhere else, interpreted with the leaf or slot operand read
// at run time (a lane's handler work is a handful of instructions, so a
// compact dispatch matters more than specialised handlers).
//
// Lanes enumerate units u = position * 2^(nvars*n) + valuation in order, so
// the lowest failing lane of the lowest failing block holds the least
// (position, valuation) and its lowest failing world the least key.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "census_kernels.h"
#include "kripke_internal.h"

namespace kripke {
namespace {

__device__ __forceinline__ uint64_t rl64(uint64_t x, int lane) {
  uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, lane);
  uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

struct Lane {
  uint32_t succ[kWorldMaskMaxN];
  uint32_t full, any_succ, val;
  int n, nvars;
};

__device__ __forceinline__ uint32_t leaf_mask(const Lane& l, uint32_t leaf) {
  if (leaf < L_NVAR0) return (l.val >> (leaf * l.n)) & l.full;
  if (leaf < L_SUCC) return ~(l.val >> ((leaf - L_NVAR0) * l.n)) & l.full;
  if (leaf == L_SUCC) return l.any_succ;
  if (leaf == L_DEAD) return ~l.any_succ & l.full;
  return leaf == L_TOP ? l.full : 0u;
}

// Rows beyond n are empty, so both loops run over all kWorldMaskMaxN rows with
// constant indices (registers, not scratch) and the result is cut to n bits.
__device__ __forceinline__ uint32_t box(const Lane& l, uint32_t t) {
  uint32_t r = 0;
  const uint32_t nt = ~t & l.full;
#pragma unroll
  for (int w = 0; w < kWorldMaskMaxN; ++w) r |= (uint32_t)((l.succ[w] & nt) == 0) << w;
  return r & l.full;
}

__device__ __forceinline__ uint32_t dia(const Lane& l, uint32_t t) {
  uint32_t r = 0;
#pragma unroll
  for (int w = 0; w < kWorldMaskMaxN; ++w) r |= (uint32_t)((l.succ[w] & t) != 0) << w;
  return r;
}

// Stack slots with constant indices (the slot number is wave-uniform).
__device__ __forceinline__ void slot_set(uint32_t (&stk)[kMaxSlots], uint32_t d, uint32_t x) {
#pragma unroll
  for (int k = 0; k < kMaxSlots; ++k)
    if ((uint32_t)k == d) stk[k] = x;
}
__device__ __forceinline__ uint32_t slot_get(const uint32_t (&stk)[kMaxSlots], uint32_t d) {
  uint32_t x = 0;
#pragma unroll
  for (int k = 0; k < kMaxSlots; ++k)
    if ((uint32_t)k == d) x = stk[k];
  return x;
}

__device__ __forceinline__ uint32_t run(const Lane& l, const uint8_t* prog) {
  uint32_t acc = 0, stk[kMaxSlots];
  for (int i = 0;; ++i) {
    const uint32_t op = __builtin_amdgcn_readfirstlane(prog[i]);  // wave-uniform
    if (op == U_END) return acc;
    if (op < U_AND_L) {
      acc = leaf_mask(l, op - U_LOAD);
    } else if (op < U_OR_L) {
      acc &= leaf_mask(l, op - U_AND_L);
    } else if (op < U_IFF_L) {
      acc |= leaf_mask(l, op - U_OR_L);
    } else if (op < U_BOX) {
      acc = ~(acc ^ leaf_mask(l, op - U_IFF_L)) & l.full;
    } else if (op == U_BOX) {
      acc = box(l, acc);
    } else if (op == U_DIA) {
      acc = dia(l, acc);
    } else if (op < U_AND_S) {
      slot_set(stk, op - U_SAVE, acc);
    } else if (op < U_OR_S) {
      acc &= slot_get(stk, op - U_AND_S);
    } else if (op < U_IFF_S) {
      acc |= slot_get(stk, op - U_OR_S);
    } else if (op < U_DIA_L) {
      acc = ~(acc ^ slot_get(stk, op - U_IFF_S)) & l.full;
    } else if (op < U_BOX_L) {
      acc = dia(l, leaf_mask(l, op - U_DIA_L));
    } else if (op < U_MM) {
      acc = box(l, leaf_mask(l, op - U_BOX_L));
    } else {
      const uint32_t mm = op - U_MM;
      acc = (mm >> 1) ? dia(l, acc) : box(l, acc);
      acc = (mm & 1) ? dia(l, acc) : box(l, acc);
    }
  }
}

__global__ __launch_bounds__(256) void split_worldmask(WorldMaskArgs a) {
  __shared__ uint8_t sprog[4][kMaxMicro + 8];
  const int lane = threadIdx.x & 63;
  uint8_t* prog = sprog[threadIdx.x >> 6];
  const uint64_t nval = 1ull << (a.nvars * a.n);
  const uint64_t units = a.nframes * nval;
  const uint64_t nblocks = (units + 63) >> 6;
  Lane l;
  l.n = (int)a.n;
  l.nvars = (int)a.nvars;
  l.full = a.n >= 32 ? ~0u : (1u << a.n) - 1u;

  for (;;) {
    uint64_t item = 0;
    if (lane == 0) item = atomicAdd(a.queue, 1ull);
    item = rl64(item, 0);
    if (item >= a.total_items) break;
    const uint32_t f = a.order[item / a.items_per_pair];
    const uint64_t b0 = (item % a.items_per_pair) * a.blocks_per_item;
    const uint64_t b1 = b0 + a.blocks_per_item < nblocks ? b0 + a.blocks_per_item : nblocks;
    unsigned long long* key_out = a.out_key + f;
    // skip work that starts beyond the pair's best key
    uint64_t known = __hip_atomic_load(key_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    known = rl64(known, 0);
    if (known != ~0ull && (known >> (a.nvars * a.n + 4)) < (b0 << 6) / nval) continue;

    const uint32_t p0 = a.uoff[f], pl = a.uoff[f + 1] - p0;
    for (uint32_t i = lane; i < pl; i += 64) prog[i] = a.ucode[p0 + i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    uint64_t key = ~0ull;
    for (uint64_t blk = b0; blk < b1 && key == ~0ull; ++blk) {
      const uint64_t u = (blk << 6) + lane;
      const bool valid = u < units;
      const uint64_t pos = valid ? u / nval : 0;
      l.val = (uint32_t)(valid ? u % nval : 0);
      const uint32_t* s = a.frames + pos * a.n;
      l.any_succ = 0;
#pragma unroll
      for (int w = 0; w < kWorldMaskMaxN; ++w) {
        const bool row = (uint32_t)w < a.n;
        const uint32_t x = s[row ? w : 0];  // never read past the frame's n rows
        l.succ[w] = row ? x & l.full : 0u;
        l.any_succ |= (uint32_t)(l.succ[w] != 0) << w;
      }
      const uint32_t truth = run(l, prog);
      const uint32_t fail = valid ? (~truth & l.full) : 0u;
      const uint64_t bal = __ballot(fail != 0);
      if (bal) {
        const int fl = __builtin_ctzll(bal);
        const uint64_t lk = (pos << (a.nvars * a.n + 4)) | ((uint64_t)l.val << 4) |
                            (uint64_t)__builtin_ctz(fail | 0x80000000u);
        key = rl64(lk, fl);
      }
    }
    if (lane == 0 && key != ~0ull) atomicMin(key_out, (unsigned long long)key);
  }
}

}  // namespace

hipError_t launch_split_worldmask(const WorldMaskArgs& a, int grid, hipStream_t s) {
  if (a.n < 1 || a.n > (uint32_t)kWorldMaskMaxN || a.nvars * a.n > 24) return hipErrorInvalidValue;
  hipLaunchKernelGGL(split_worldmask, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace kripke
