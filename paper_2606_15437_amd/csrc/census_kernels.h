// Launch interface between the C ABI layer and the census kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace kripke {

enum Mode : int {
  M_RANGE_K = 0,   // positions are raw frame indices
  M_RANGE_T = 1,   // positions enumerate reflexive frames in index order
  M_LIST_IDX = 2,  // positions index a device list of frame indices
  M_LIST_SUCC = 3  // positions index a device list of successor-mask rows
};

struct CensusArgs {
  const uint8_t* ucode;        // compiled programs, each padded to 4 bytes
  const uint32_t* uoff;        // byte offsets [nformulas + 1], multiples of 4
  const uint32_t* order;       // processing order of the formulas (costliest first)
  uint32_t nformulas;
  int mode;
  uint64_t pos_begin;          // first position of the scan
  uint64_t npos;               // number of positions
  const uint64_t* list_idx;    // M_LIST_IDX
  const uint32_t* list_succ;   // M_LIST_SUCC, [positions][n]
  uint64_t blocks_per_item;    // 64-unit blocks per work item
  uint64_t items_per_formula;
  uint64_t total_items;
  unsigned long long* queue;   // work-item counter, zeroed before launch
  unsigned long long* out_key; // first key of formula f at out_key[f * out_stride]
  unsigned long long* out_cnt; // fail count of formula f (nullptr: not counted)
  uint32_t out_stride;         // in 64-bit words
  uint32_t decide;             // stop at the first countermodel
  uint32_t key_pos;            // key frame field = position instead of frame index
};

// List modes 2 and 3 scan a group of up to this many formulas per work item,
// so each block's frame rows are loaded and decoded once per group.
constexpr uint32_t kListGroupMax = 4;

// Arguments of the wave-uniform-frame kernel.  Positions are frame indices
// (mode 0, class K), ranks of reflexive frames (mode 1, class T) or indices
// into a list of successor rows (mode 2: one list frame per block; mode 3:
// two, one per half-wave); a block holds 2^fast_block_log2() consecutive
// positions.
struct FastArgs {
  const uint8_t* ucode;
  const uint32_t* uoff;
  const uint32_t* order;
  uint32_t nformulas;
  uint64_t pos_begin, pos_end;  // scanned positions [pos_begin, pos_end)
  uint64_t blk_begin, nblk;     // blocks covering them
  uint64_t blocks_per_item, items_per_formula, total_items;
  unsigned long long* queue;
  const uint32_t* levels;       // fused: 2-bit class level per frame, 16 per word
  unsigned long long* out_key;  // class-0 row; class k at + k * class_stride
  unsigned long long* out_cnt;
  uint32_t out_stride;
  uint64_t class_stride;
  uint32_t decide;
  const uint32_t* list_succ;    // modes 2, 3: successor rows [positions][n]
  uint32_t group;               // modes 2, 3: formulas per work item (1..kListGroupMax)
  uint32_t* valid_bits;         // optional frame-validity maps [nformulas][valid_words],
  uint64_t valid_words;         // bit p = no countermodel on position p (mode 0)
};

bool fast_available(int n, int nvars, int ls, int mode, bool fused);
int fast_block_log2(int n, int nvars, int ls, int mode);
int fast_stack_slots(int n, int nvars, int ls, int mode, bool fused);
hipError_t launch_fast(const FastArgs& a, int n, int nvars, int ls, int mode, bool fused, int grid,
                       hipStream_t s);
int fast_blocks_per_cu(int n, int nvars, int ls, int mode, bool fused);
hipError_t launch_levels(int n, uint32_t* levels, hipStream_t s);
uint64_t refl_frame_host(uint64_t j, int n);
hipError_t run_calibration(int cus, uint32_t iters, double* lane_ops_per_s, hipStream_t s);

// Signature bits: formulas x groups of 64 pointed-model samples of one n.
struct SigArgs {
  const uint8_t* ucode;
  const uint32_t* uoff;
  uint32_t nformulas;
  const uint64_t* samples;  // n << 60 | frame << 24 | val << 4 | world
  const uint32_t* groups;   // indices of the 64-sample groups with this n
  uint32_t ngroups;
  uint32_t words;           // signature words per formula (all groups)
  unsigned long long* sig;  // [nformulas][words]
};
hipError_t launch_signatures(const SigArgs& a, int n, int nvars, hipStream_t s);

// Candidate pairs: the k nearest formulas of each formula by signature
// Hamming distance, then the unordered pairs in canonical order.
hipError_t launch_knn(const uint64_t* sig, uint32_t nformulas, uint32_t words, uint32_t k,
                      uint32_t* nbr, hipStream_t s);
int knn_pairs_canonical(const uint32_t* nbr, uint32_t nformulas, uint32_t k, uint64_t* pairs,
                        uint64_t* npairs, hipStream_t s);
hipError_t launch_pair_hamming(const uint64_t* sig, uint32_t words, const uint64_t* pairs,
                               uint64_t npairs, uint32_t* dist, hipStream_t s);
int select_top(const float* scores, uint64_t n, uint64_t budget, uint64_t* idx, hipStream_t s);

hipError_t launch_census(const CensusArgs& a, int n, int nvars, int grid, hipStream_t s);

// Split search with world-set bitmasks (large frames): pair f's biconditional
// program at ucode[uoff[f] .. uoff[f+1]), frames = successor rows [nframes][n].
constexpr int kWorldMaskMaxN = 16;
struct WorldMaskArgs {
  const uint8_t* ucode;
  const uint32_t* uoff;
  const uint32_t* order;
  const uint32_t* frames;
  uint64_t nframes;
  uint32_t n, nvars;
  uint64_t blocks_per_item, items_per_pair, total_items;
  unsigned long long* queue;
  unsigned long long* out_key;  // [npairs]
};
hipError_t launch_split_worldmask(const WorldMaskArgs& a, int grid, hipStream_t s);
int census_blocks_per_cu(int n, int nvars);
hipError_t launch_init(unsigned long long* key, unsigned long long* cnt, uint32_t stride,
                       uint32_t count, unsigned long long* queue, hipStream_t s);
// rows[r][0..words) = value[r] for r < nrows
hipError_t launch_fill_rows(uint32_t* rows, uint64_t words, const uint32_t* value, uint32_t nrows,
                            hipStream_t s);
hipError_t launch_class_list(int n, int level, uint32_t* counts, uint64_t* total, uint64_t* list,
                             hipStream_t s);
uint64_t t_frame_host(uint64_t j, int n);

}  // namespace kripke
