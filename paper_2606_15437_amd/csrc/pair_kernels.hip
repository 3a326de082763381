// Candidate-pair construction and ranking for the learned proposal.
//
// A formula's signature is its truth bits at a fixed sample of small pointed
// models.  Candidate pairs are, for every formula, its k nearest formulas by
// signature Hamming distance (ties to the smaller index), taken as unordered
// pairs in canonical (i < j) order.  Rankings select the top `budget` pairs
// by score, ties to the earlier canonical position (a stable sort).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cstdint>

#include "census_kernels.h"

namespace kripke {
namespace {

constexpr int kMaxKnnFormulas = 16384;  // distances of one row held in LDS
constexpr int kMaxBits = 8192;          // signature bits (histogram bins)

// One block per formula i: distances to every j in LDS, a histogram to find
// the k-th smallest distance T, then the j with d < T plus the smallest-index
// j with d == T, emitted in increasing j.
__global__ __launch_bounds__(256) void knn_kernel(const uint64_t* sig, uint32_t nf, uint32_t words,
                                                  uint32_t k, uint32_t* nbr) {
  __shared__ uint16_t dist[kMaxKnnFormulas];
  __shared__ uint32_t hist[kMaxBits + 1];
  __shared__ uint64_t row[kMaxBits / 64];
  __shared__ uint32_t wave_cnt[4][2];
  __shared__ uint32_t thresh, need_eq, run_eq, run_out;
  const uint32_t i = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (uint32_t w = t; w < words; w += 256) row[w] = sig[(uint64_t)i * words + w];
  for (uint32_t b = t; b <= words * 64; b += 256) hist[b] = 0;
  __syncthreads();
  for (uint32_t j = t; j < nf; j += 256) {
    uint32_t d = 0;
    const uint64_t* sj = sig + (uint64_t)j * words;
    for (uint32_t w = 0; w < words; ++w) d += __builtin_popcountll(row[w] ^ sj[w]);
    dist[j] = (uint16_t)d;
    if (j != i) atomicAdd(&hist[d], 1u);
  }
  __syncthreads();
  if (t == 0) {
    uint32_t below = 0, b = 0;
    while (below + hist[b] < k) below += hist[b++];
    thresh = b;
    need_eq = k - below;
    run_eq = run_out = 0;
  }
  __syncthreads();
  const uint32_t T = thresh, need = need_eq;
  for (uint32_t base = 0; base < nf; base += 256) {
    const uint32_t j = base + t;
    const bool ok = j < nf && j != i;
    const bool lt = ok && dist[j] < T;
    const bool eq = ok && dist[j] == T;
    const uint64_t beq = __ballot(eq);
    if (lane == 0) wave_cnt[wv][0] = __builtin_popcountll(beq);
    __syncthreads();
    uint32_t eq_before = run_eq;
    for (int x = 0; x < wv; ++x) eq_before += wave_cnt[x][0];
    eq_before += __builtin_popcountll(beq & ((1ull << lane) - 1ull));
    const bool take = lt || (eq && eq_before < need);
    const uint64_t btake = __ballot(take);
    if (lane == 0) wave_cnt[wv][1] = __builtin_popcountll(btake);
    __syncthreads();
    uint32_t pos = run_out;
    for (int x = 0; x < wv; ++x) pos += wave_cnt[x][1];
    pos += __builtin_popcountll(btake & ((1ull << lane) - 1ull));
    if (take) nbr[(uint64_t)i * k + pos] = j;
    __syncthreads();
    if (t == 0) {
      run_eq += wave_cnt[0][0] + wave_cnt[1][0] + wave_cnt[2][0] + wave_cnt[3][0];
      run_out += wave_cnt[0][1] + wave_cnt[1][1] + wave_cnt[2][1] + wave_cnt[3][1];
    }
    __syncthreads();
  }
}

__global__ void pair_keys(const uint32_t* nbr, uint32_t nf, uint32_t k, uint64_t* keys) {
  const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= (uint64_t)nf * k) return;
  const uint64_t i = x / k, j = nbr[x];
  keys[x] = i < j ? (i << 32) | j : (j << 32) | i;
}

__global__ void pair_hamming(const uint64_t* sig, uint32_t words, const uint64_t* pairs,
                             uint64_t npairs, uint32_t* dist) {
  const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= npairs) return;
  const uint64_t i = pairs[x] >> 32, j = pairs[x] & 0xFFFFFFFFu;
  uint32_t d = 0;
  for (uint32_t w = 0; w < words; ++w)
    d += __builtin_popcountll(sig[i * words + w] ^ sig[j * words + w]);
  dist[x] = d;
}

__global__ void iota_u64(uint64_t* v, uint64_t n) {
  const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < n) v[x] = x;
}

// Order-preserving map of a float score to an unsigned key (larger score,
// larger key; -0 and +0 equal).
__global__ void score_keys(const float* s, uint64_t n, uint32_t* keys) {
  const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  float f = s[x];
  if (f == 0.0f) f = 0.0f;
  const uint32_t u = __float_as_uint(f);
  keys[x] = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

uint32_t blocks_for(uint64_t n) { return (uint32_t)((n + 255) / 256); }

}  // namespace

hipError_t launch_knn(const uint64_t* sig, uint32_t nformulas, uint32_t words, uint32_t k,
                      uint32_t* nbr, hipStream_t s) {
  if (nformulas > (uint32_t)kMaxKnnFormulas || words * 64 > (uint32_t)kMaxBits || k == 0 ||
      k >= nformulas)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(knn_kernel, dim3(nformulas), dim3(256), 0, s, sig, nformulas, words, k, nbr);
  return hipGetLastError();
}

// Sort the directed neighbour entries as (min, max) keys and drop
// duplicates: the canonical (i < j) order of the unordered candidate pairs.
int knn_pairs_canonical(const uint32_t* nbr, uint32_t nformulas, uint32_t k, uint64_t* pairs,
                        uint64_t* npairs, hipStream_t s) {
  const uint64_t n = (uint64_t)nformulas * k;
  uint64_t *keys = nullptr, *sorted = nullptr;
  void* tmp = nullptr;
  size_t tmp_sort = 0, tmp_uniq = 0;
  int rc = 0;  // 0, -5 (allocation failed) or -4 (a HIP or hipCUB call failed)
  if (hipMallocAsync((void**)&keys, n * 8, s) != hipSuccess ||
      hipMallocAsync((void**)&sorted, n * 8, s) != hipSuccess) {
    rc = -5;
  } else {
    hipLaunchKernelGGL(pair_keys, dim3(blocks_for(n)), dim3(256), 0, s, nbr, nformulas, k, keys);
    if (hipGetLastError() != hipSuccess ||
        hipcub::DeviceRadixSort::SortKeys(nullptr, tmp_sort, keys, sorted, (int)n, 0, 64, s) !=
            hipSuccess ||
        hipcub::DeviceSelect::Unique(nullptr, tmp_uniq, sorted, pairs, npairs, (int)n, s) !=
            hipSuccess)
      rc = -4;
  }
  if (rc == 0) {
    const size_t tb = tmp_sort > tmp_uniq ? tmp_sort : tmp_uniq;
    size_t b1 = tb, b2 = tb;
    if (hipMallocAsync(&tmp, tb, s) != hipSuccess)
      rc = -5;
    else if (hipcub::DeviceRadixSort::SortKeys(tmp, b1, keys, sorted, (int)n, 0, 64, s) !=
                 hipSuccess ||
             hipcub::DeviceSelect::Unique(tmp, b2, sorted, pairs, npairs, (int)n, s) != hipSuccess)
      rc = -4;
  }
  // stream-ordered frees after the work that uses the buffers
  if (tmp) (void)hipFreeAsync(tmp, s);
  if (keys) (void)hipFreeAsync(keys, s);
  if (sorted) (void)hipFreeAsync(sorted, s);
  return rc;
}

hipError_t launch_pair_hamming(const uint64_t* sig, uint32_t words, const uint64_t* pairs,
                               uint64_t npairs, uint32_t* dist, hipStream_t s) {
  if (npairs == 0) return hipSuccess;
  hipLaunchKernelGGL(pair_hamming, dim3(blocks_for(npairs)), dim3(256), 0, s, sig, words, pairs,
                     npairs, dist);
  return hipGetLastError();
}

// Indices of the `budget` highest scores, highest first; equal scores keep
// their input order (the radix sort is stable).
int select_top(const float* scores, uint64_t n, uint64_t budget, uint64_t* idx, hipStream_t s) {
  uint32_t *keys = nullptr, *keys_out = nullptr;
  uint64_t *vals = nullptr, *vals_out = nullptr;
  void* tmp = nullptr;
  size_t tb = 0;
  int rc = 0;  // 0, -5 (allocation failed) or -4 (a HIP or hipCUB call failed)
  if (hipMallocAsync((void**)&keys, n * 4, s) != hipSuccess ||
      hipMallocAsync((void**)&keys_out, n * 4, s) != hipSuccess ||
      hipMallocAsync((void**)&vals, n * 8, s) != hipSuccess ||
      hipMallocAsync((void**)&vals_out, n * 8, s) != hipSuccess) {
    rc = -5;
  } else {
    hipLaunchKernelGGL(score_keys, dim3(blocks_for(n)), dim3(256), 0, s, scores, n, keys);
    hipLaunchKernelGGL(iota_u64, dim3(blocks_for(n)), dim3(256), 0, s, vals, n);
    if (hipGetLastError() != hipSuccess ||
        hipcub::DeviceRadixSort::SortPairsDescending(nullptr, tb, keys, keys_out, vals, vals_out,
                                                     (int)n, 0, 32, s) != hipSuccess)
      rc = -4;
  }
  if (rc == 0) {
    if (hipMallocAsync(&tmp, tb, s) != hipSuccess)
      rc = -5;
    else if (hipcub::DeviceRadixSort::SortPairsDescending(tmp, tb, keys, keys_out, vals, vals_out,
                                                          (int)n, 0, 32, s) != hipSuccess ||
             hipMemcpyAsync(idx, vals_out, (budget < n ? budget : n) * 8,
                            hipMemcpyDeviceToDevice, s) != hipSuccess)
      rc = -4;
  }
  // stream-ordered frees after the work that uses the buffers
  if (tmp) (void)hipFreeAsync(tmp, s);
  if (keys) (void)hipFreeAsync(keys, s);
  if (keys_out) (void)hipFreeAsync(keys_out, s);
  if (vals) (void)hipFreeAsync(vals, s);
  if (vals_out) (void)hipFreeAsync(vals_out, s);
  return rc;
}

}  // namespace kripke
