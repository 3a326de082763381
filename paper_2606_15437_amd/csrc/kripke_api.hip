// C ABI of libkripke.so: validation, program compilation, frame-class lists,
// work partitioning, plans with hipGraph replay, and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/kripke.h"
#include "census_kernels.h"
#include "mlp_kernels.h"
#include "kripke_internal.h"

using namespace kripke;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define KR_HIP(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(KRIPKE_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
  } while (0)

// ------------------------------------------------------------ batches
struct MicroBatch {
  std::vector<uint8_t> code;      // programs, each padded to 8 bytes with U_END
  std::vector<uint32_t> off;      // [count + 1]
  std::vector<uint32_t> order;    // costliest first
  std::vector<int> is_const;
  uint64_t cost_total = 0;
  int max_slots = 0;
  std::vector<int> slots;         // stack slots per formula
};

// Compile programs [lo, hi) of a batch into a part of a MicroBatch (micro-op
// code with local offsets).  Runs on worker threads: it reports a failure
// through rc/err instead of the thread-local error slot.
struct BatchPart {
  std::vector<uint8_t> code;
  std::vector<uint32_t> end;  // end offset of each program within `code`
  std::vector<int> is_const, slots;
  std::vector<uint64_t> cost;
  int max_slots = 0;
  int rc = KRIPKE_OK;
  std::string err;
};

void compile_part(const uint8_t* code, const uint32_t* offsets, uint32_t lo, uint32_t hi,
                  uint32_t nvars, int n, bool pairs, BatchPart* part) {
  for (uint32_t i = lo; i < hi; ++i) {
    Compiled c;
    std::string err;
    int rc;
    if (pairs) {
      const uint32_t a0 = offsets[2 * i], a1 = offsets[2 * i + 1], b1 = offsets[2 * i + 2];
      rc = compile_iff(code + a0, a1 - a0, code + a1, b1 - a1, nvars, &c, &err);
    } else {
      rc = compile_program(code + offsets[i], offsets[i + 1] - offsets[i], nvars, &c, &err);
    }
    if (rc == KRIPKE_OK && c.micro.size() + 3 > (size_t)kMaxMicro) {
      // the kernels stage each program in a fixed per-wave LDS slot
      rc = KRIPKE_ELIMIT;
      err = "compiled program too long";
    }
    if (rc != KRIPKE_OK) {
      part->rc = rc;
      part->err = (pairs ? "pair " : "formula ") + std::to_string(i) + ": " + err;
      return;
    }
    part->code.insert(part->code.end(), c.micro.begin(), c.micro.end());
    while (part->code.size() % 8) part->code.push_back(U_END);  // kernels fetch 8 ops at a time
    part->end.push_back((uint32_t)part->code.size());
    part->is_const.push_back(c.is_const);
    part->max_slots = std::max(part->max_slots, c.slots);
    part->slots.push_back(c.slots);
    part->cost.push_back((uint64_t)c.modal * n * n + (uint64_t)(c.binary + c.loads + c.saves) * n +
                         8);
  }
}

int compile_batch(const uint8_t* code, const uint32_t* offsets, uint32_t count, uint32_t nvars,
                  int n, bool pairs, MicroBatch* mb) {
  if (!code || !offsets) return fail(KRIPKE_EINVAL, "null code/offsets");
  if (offsets[0] != 0) return fail(KRIPKE_EINVAL, "offsets[0] must be 0");
  const uint32_t progs = pairs ? 2 * count : count;
  for (uint32_t i = 0; i < progs; ++i)
    if (offsets[i + 1] < offsets[i]) return fail(KRIPKE_EINVAL, "offsets must be non-decreasing");
  // large batches compile on several host threads, each over a contiguous
  // range; the parts are joined in order, so the result does not depend on
  // the thread count
  const uint32_t hw = std::max(1u, std::thread::hardware_concurrency());
  const uint32_t nparts = count >= 8192 ? std::min<uint32_t>(std::min<uint32_t>(hw, 32),
                                                             count / 4096)
                                        : 1;
  std::vector<BatchPart> parts(nparts);
  if (nparts == 1) {
    compile_part(code, offsets, 0, count, nvars, n, pairs, &parts[0]);
  } else {
    std::vector<std::thread> th;
    for (uint32_t t = 0; t < nparts; ++t)
      th.emplace_back(compile_part, code, offsets, (uint32_t)((uint64_t)count * t / nparts),
                      (uint32_t)((uint64_t)count * (t + 1) / nparts), nvars, n, pairs, &parts[t]);
    for (auto& x : th) x.join();
  }
  for (const BatchPart& part : parts)  // the first failing program in batch order
    if (part.rc != KRIPKE_OK) return fail(part.rc, part.err);
  mb->code.clear();
  mb->off.assign(1, 0);
  mb->is_const.clear();
  mb->slots.clear();
  mb->max_slots = 0;
  mb->cost_total = 0;
  std::vector<uint64_t> cost;
  cost.reserve(count);
  for (const BatchPart& part : parts) {
    const uint32_t base = (uint32_t)mb->code.size();
    mb->code.insert(mb->code.end(), part.code.begin(), part.code.end());
    for (uint32_t e : part.end) mb->off.push_back(base + e);
    mb->is_const.insert(mb->is_const.end(), part.is_const.begin(), part.is_const.end());
    mb->slots.insert(mb->slots.end(), part.slots.begin(), part.slots.end());
    mb->max_slots = std::max(mb->max_slots, part.max_slots);
    cost.insert(cost.end(), part.cost.begin(), part.cost.end());
  }
  for (uint64_t c : cost) mb->cost_total += c;
  mb->order.resize(count);
  std::iota(mb->order.begin(), mb->order.end(), 0u);
  std::stable_sort(mb->order.begin(), mb->order.end(),
                   [&](uint32_t x, uint32_t y) { return cost[x] > cost[y]; });
  return KRIPKE_OK;
}

int check_sizes(uint32_t n, uint32_t nvars, int max_n) {
  if (n < 1 || (int)n > max_n)
    return fail(KRIPKE_ELIMIT, "n must be in 1.." + std::to_string(max_n));
  if (nvars > 4) return fail(KRIPKE_ELIMIT, "nvars must be <= 4");
  if (n * n + nvars * n + 4 > 64) return fail(KRIPKE_ELIMIT, "key does not fit 64 bits");
  return KRIPKE_OK;
}

// ------------------------------------------------------- device state
struct ClassList {
  uint64_t* d_list = nullptr;
  std::vector<uint64_t> host;
};

struct DeviceState {
  int cus = 0;
  std::map<std::pair<int, int>, ClassList> lists;  // (n, level)
  std::map<int, uint32_t*> levels;                 // n -> 2-bit class level per frame
};

std::mutex g_mu;
std::map<int, DeviceState> g_dev;

int device_state(DeviceState** out) {
  int dev = 0;
  KR_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceState& ds = g_dev[dev];
  if (ds.cus == 0) KR_HIP(hipDeviceGetAttribute(&ds.cus, hipDeviceAttributeMultiprocessorCount, dev));
  *out = &ds;
  return KRIPKE_OK;
}

// Ordered list of the frames on n worlds whose class level is >= level,
// built once per device on an internal stream and kept until exit.
int class_list(DeviceState* ds, int n, int level, const ClassList** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(n, level);
  auto it = ds->lists.find(key);
  if (it != ds->lists.end()) {
    *out = &it->second;
    return KRIPKE_OK;
  }
  const uint64_t nframes = 1ull << (n * n);
  const uint32_t nblocks = (uint32_t)((nframes + 255) / 256);
  hipStream_t s;
  KR_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  uint32_t* counts = nullptr;
  uint64_t* total = nullptr;
  KR_HIP(hipMalloc(&counts, sizeof(uint32_t) * nblocks));
  KR_HIP(hipMalloc(&total, sizeof(uint64_t)));
  KR_HIP(launch_class_list(n, level, counts, total, nullptr, s));
  uint64_t h_total = 0;
  KR_HIP(hipMemcpyAsync(&h_total, total, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  KR_HIP(hipStreamSynchronize(s));
  ClassList cl;
  KR_HIP(hipMalloc(&cl.d_list, sizeof(uint64_t) * (h_total ? h_total : 1)));
  KR_HIP(launch_class_list(n, level, counts, total, cl.d_list, s));
  cl.host.resize(h_total);
  if (h_total)
    KR_HIP(hipMemcpyAsync(cl.host.data(), cl.d_list, sizeof(uint64_t) * h_total,
                          hipMemcpyDeviceToHost, s));
  KR_HIP(hipStreamSynchronize(s));
  KR_HIP(hipFree(counts));
  KR_HIP(hipFree(total));
  KR_HIP(hipStreamDestroy(s));
  auto res = ds->lists.emplace(key, std::move(cl));
  *out = &res.first->second;
  return KRIPKE_OK;
}

// Class level of every frame on n <= 5 worlds, built once per device.
int level_table(DeviceState* ds, int n, const uint32_t** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = ds->levels.find(n);
  if (it != ds->levels.end()) {
    *out = it->second;
    return KRIPKE_OK;
  }
  const uint64_t nwords = ((1ull << (n * n)) + 15) / 16;
  uint32_t* d = nullptr;
  hipStream_t s;
  KR_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  KR_HIP(hipMalloc(&d, nwords * sizeof(uint32_t)));
  KR_HIP(launch_levels(n, d, s));
  KR_HIP(hipStreamSynchronize(s));
  KR_HIP(hipStreamDestroy(s));
  ds->levels[n] = d;
  *out = d;
  return KRIPKE_OK;
}

// Least reflexive-enumeration position whose frame index is >= f.
uint64_t t_rank(uint64_t f, int n) {
  uint64_t lo = 0, hi = 1ull << (n * n - n);
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (t_frame_host(mid, n) < f) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Work partition of one scan: positions x 2^(V-5) valuation words in blocks
// of 64 units, split into items so every wave gets several.
struct Scan {
  int mode = M_RANGE_K;
  uint64_t pos_begin = 0, npos = 0;
  const uint64_t* list_idx = nullptr;
  const uint32_t* list_succ = nullptr;
};

void partition(const Scan& sc, int n, int nvars, uint32_t nformulas, int grid, CensusArgs* a) {
  const int V = n * nvars;
  const int wlog = V > 5 ? V - 5 : 0;
  const uint64_t units = sc.npos << wlog;
  const uint64_t nblocks = std::max<uint64_t>(1, (units + 63) / 64);
  const uint64_t waves = (uint64_t)grid * 4;
  const uint64_t target = std::max<uint64_t>(16 * waves, nformulas);
  uint64_t bpi = std::max<uint64_t>(1, (nblocks * nformulas + target - 1) / target);
  bpi = std::min<uint64_t>(bpi, 1ull << 20);
  a->mode = sc.mode;
  a->pos_begin = sc.pos_begin;
  a->npos = sc.npos;
  a->list_idx = sc.list_idx;
  a->list_succ = sc.list_succ;
  a->blocks_per_item = bpi;
  a->items_per_formula = (nblocks + bpi - 1) / bpi;
  a->total_items = a->items_per_formula * nformulas;
  a->nformulas = nformulas;
}

int grid_for(DeviceState* ds, int n, int nvars, uint64_t total_items) {
  const int per_cu = census_blocks_per_cu(n, nvars);
  uint64_t g = (uint64_t)ds->cus * per_cu;
  g = std::min<uint64_t>(g, std::max<uint64_t>(1, (total_items + 3) / 4));
  return (int)g;
}

// Resolve the positions scanned for class `cls` over raw frames [f0, f1).
int make_scan(DeviceState* ds, int n, int cls, uint64_t f0, uint64_t f1, Scan* sc) {
  if (cls == KRIPKE_K) {
    sc->mode = M_RANGE_K;
    sc->pos_begin = f0;
    sc->npos = f1 - f0;
  } else if (cls == KRIPKE_T) {
    sc->mode = M_RANGE_T;
    sc->pos_begin = t_rank(f0, n);
    sc->npos = t_rank(f1, n) - sc->pos_begin;
  } else {
    if (n > 5) return fail(KRIPKE_ELIMIT, "S4/S5 census supports n <= 5");
    const ClassList* cl = nullptr;
    int rc = class_list(ds, n, cls, &cl);
    if (rc) return rc;
    auto lo = std::lower_bound(cl->host.begin(), cl->host.end(), f0);
    auto hi = std::lower_bound(cl->host.begin(), cl->host.end(), f1);
    sc->mode = M_LIST_IDX;
    sc->list_idx = cl->d_list;
    sc->pos_begin = (uint64_t)(lo - cl->host.begin());
    sc->npos = (uint64_t)(hi - lo);
  }
  return KRIPKE_OK;
}

// Device copies of a compiled batch.
struct DeviceBatch {
  uint8_t* ucode = nullptr;
  uint32_t* uoff = nullptr;
  uint32_t* order = nullptr;
  unsigned long long* queue = nullptr;
};

int upload(const MicroBatch& mb, DeviceBatch* db, int nqueues, hipStream_t s) {
  KR_HIP(hipMallocAsync((void**)&db->ucode, mb.code.size(), s));
  KR_HIP(hipMallocAsync((void**)&db->uoff, mb.off.size() * 4, s));
  KR_HIP(hipMallocAsync((void**)&db->order, mb.order.size() * 4 + 4, s));
  KR_HIP(hipMallocAsync((void**)&db->queue, 8 * nqueues, s));
  KR_HIP(hipMemcpyAsync(db->ucode, mb.code.data(), mb.code.size(), hipMemcpyHostToDevice, s));
  KR_HIP(hipMemcpyAsync(db->uoff, mb.off.data(), mb.off.size() * 4, hipMemcpyHostToDevice, s));
  KR_HIP(hipMemcpyAsync(db->order, mb.order.data(), mb.order.size() * 4, hipMemcpyHostToDevice, s));
  // the host vectors die with the caller's frame: wait for the copies
  KR_HIP(hipStreamSynchronize(s));
  return KRIPKE_OK;
}

int release(DeviceBatch* db, hipStream_t s) {
  KR_HIP(hipFreeAsync(db->ucode, s));
  KR_HIP(hipFreeAsync(db->uoff, s));
  KR_HIP(hipFreeAsync(db->order, s));
  KR_HIP(hipFreeAsync(db->queue, s));
  return KRIPKE_OK;
}

int enqueue_scan(DeviceState* ds, const DeviceBatch& db, const Scan& sc, int n, int nvars,
                 uint32_t nformulas, unsigned long long* key, unsigned long long* cnt,
                 uint32_t stride, bool decide, bool key_pos, unsigned long long* queue,
                 hipStream_t s, uint32_t init_first = 0) {
  CensusArgs a{};
  a.ucode = db.ucode;
  a.uoff = db.uoff;
  a.order = db.order;
  partition(sc, n, nvars, nformulas, ds->cus * census_blocks_per_cu(n, nvars), &a);
  a.queue = queue;
  a.out_key = key;
  a.out_cnt = cnt;
  a.out_stride = stride;
  a.decide = decide;
  a.key_pos = key_pos;
  KR_HIP(launch_init(key + (uint64_t)stride * init_first,
                     cnt ? cnt + (uint64_t)stride * init_first : nullptr, stride, nformulas, queue,
                     s));
  if (sc.npos == 0) return KRIPKE_OK;
  KR_HIP(launch_census(a, n, nvars, grid_for(ds, n, nvars, a.total_items), s));
  return KRIPKE_OK;
}

// Preferred number of frame sets per lane (log2) for the fast kernel, or -1
// if no variant fits; KRIPKE_SETS_LOG2 overrides the default for tuning.
int pick_sets(int n, int nvars, int mode, bool fused, int max_slots) {
  const char* env = getenv("KRIPKE_SETS_LOG2");
  std::vector<int> pref = {2, 1, 0};
  if (env) pref.insert(pref.begin(), atoi(env));
  for (int ls : pref)
    if (ls >= 0 && ls <= 3 && fast_available(n, nvars, ls, mode, fused) &&
        max_slots <= fast_stack_slots(n, nvars, ls, mode, fused))
      return ls;
  return -1;
}

// Two-tier split of a batch for the fast kernel: programs whose stack need
// fits variant `ls` run in one launch, the deeper rest in a second launch
// with the widest variant that fits them.  order = tier A then tier B, each
// costliest first.
struct Tiering {
  std::vector<uint32_t> order;
  uint32_t count_a = 0;
  int ls_a = -1, ls_b = -1;
  int mode_a = -1, mode_b = -1;  // kernel mode of each tier
};

bool make_tiers(const MicroBatch& mb, int n, int nvars, int mode, bool fused, int ls,
                Tiering* t) {
  if (ls < 0 || !fast_available(n, nvars, ls, mode, fused)) return false;
  t->mode_a = t->mode_b = mode;
  t->order.clear();
  int max_b = 0;
  for (uint32_t f : mb.order)
    if (mb.slots[f] <= fast_stack_slots(n, nvars, ls, mode, fused)) t->order.push_back(f);
  t->count_a = (uint32_t)t->order.size();
  for (uint32_t f : mb.order)
    if (mb.slots[f] > fast_stack_slots(n, nvars, ls, mode, fused)) {
      t->order.push_back(f);
      max_b = std::max(max_b, mb.slots[f]);
    }
  t->ls_a = ls;
  t->ls_b = -1;
  if (t->count_a < t->order.size()) {
    // the deeper programs: the widest variant of the same mode that holds them;
    // two-frame list blocks fall back to one-frame list blocks (same keys)
    for (int m : {mode, mode == 3 ? 2 : mode})
      for (int l = 2; l >= 0 && t->ls_b < 0; --l)
        if (fast_available(n, nvars, l, m, fused) &&
            max_b <= fast_stack_slots(n, nvars, l, m, fused)) {
          t->ls_b = l;
          t->mode_b = m;
        }
    if (t->ls_b < 0) return false;
  }
  return true;
}

// Preferred tiering for a batch (env override, then widest variant first).
bool pick_tiers(const MicroBatch& mb, int n, int nvars, int mode, bool fused, Tiering* t) {
  const char* env = getenv("KRIPKE_SETS_LOG2");
  std::vector<int> pref = {2, 1, 3, 0};
  if (env) pref.insert(pref.begin(), atoi(env));
  for (int ls : pref)
    if (ls >= 0 && ls <= 3 && make_tiers(mb, n, nvars, mode, fused, ls, t)) return true;
  return false;
}

// Enqueue the fast census over positions [p0, p1) (frame indices for mode 0,
// reflexive ranks for mode 1).  With `fused`, out_key/out_cnt are the class-0
// row of a [4][nformulas] result array.
int enqueue_fast(DeviceState* ds, const DeviceBatch& db, int n, int nvars, int ls, int mode,
                 bool fused, uint32_t nformulas, uint64_t p0, uint64_t p1,
                 unsigned long long* key, unsigned long long* cnt, bool decide,
                 unsigned long long* queue, hipStream_t s, int items_per_wave = 16,
                 uint32_t init_first = 0, uint32_t order_first = 0, bool init = true,
                 uint32_t row_formulas = 0, uint32_t out_stride = 2,
                 const uint32_t* list_succ = nullptr, uint32_t* valid_bits = nullptr,
                 uint64_t valid_words = 0) {
  // row_formulas: formulas per class row of the output (the whole batch, which
  // a tier launch covers only part of); out_stride: 64-bit words between the
  // keys of consecutive formulas (2 for census results, 1 for split keys);
  // list_succ: the frame list of modes 2 and 3
  if (row_formulas == 0) row_formulas = nformulas;
  // list modes scan groups of formulas per work item and search first keys only
  uint32_t group = 1;
  if (mode >= 2) {
    if (!decide || cnt || valid_bits)
      return fail(KRIPKE_EINTERNAL, "list-mode blocks search first keys only");
    group = kListGroupMax;
    if (const char* env = getenv("KRIPKE_LIST_GROUP"))
      group = (uint32_t)std::min<long>(kListGroupMax, std::max<long>(1, atol(env)));
  }
  const uint64_t ngroups = ((uint64_t)nformulas + group - 1) / group;
  FastArgs a{};
  a.ucode = db.ucode;
  a.uoff = db.uoff;
  a.order = db.order + order_first;
  a.nformulas = nformulas;
  a.pos_begin = p0;
  a.pos_end = p1;
  const int B = fast_block_log2(n, nvars, ls, mode);
  a.blk_begin = p0 >> B;
  a.nblk = p1 > p0 ? ((p1 + (1ull << B) - 1) >> B) - a.blk_begin : 0;
  const int per_cu = fast_blocks_per_cu(n, nvars, ls, mode, fused);
  const uint64_t waves = (uint64_t)ds->cus * per_cu * 4;
  const uint64_t target = std::max<uint64_t>((uint64_t)items_per_wave * waves, ngroups);
  uint64_t bpi = std::max<uint64_t>(1, (a.nblk * ngroups + target - 1) / target);
  bpi = std::min<uint64_t>(bpi, 1ull << 16);
  a.blocks_per_item = bpi;
  a.items_per_formula = (a.nblk + bpi - 1) / bpi;  // per group in list modes
  a.total_items = a.items_per_formula * ngroups;
  a.group = group;
  a.queue = queue;
  a.out_key = key;
  a.out_cnt = cnt;
  a.out_stride = out_stride;
  a.class_stride = fused ? 2ull * row_formulas : 0;
  a.decide = decide;
  a.list_succ = list_succ;
  a.valid_bits = valid_bits;
  a.valid_words = valid_words;
  if (fused) {
    int rc = level_table(ds, n, &a.levels);
    if (rc) return rc;
  }
  if (init)
    KR_HIP(launch_init(key + (uint64_t)out_stride * init_first,
                       cnt ? cnt + (uint64_t)out_stride * init_first : nullptr, out_stride,
                       fused ? 4 * nformulas : nformulas, queue, s));
  else
    KR_HIP(launch_init(nullptr, nullptr, out_stride, 0, queue, s));
  if (a.nblk == 0 || nformulas == 0) return KRIPKE_OK;
  uint64_t grid = (uint64_t)ds->cus * per_cu;
  grid = std::min<uint64_t>(grid, std::max<uint64_t>(1, (a.total_items + 3) / 4));
  KR_HIP(launch_fast(a, n, nvars, ls, mode, fused, (int)grid, s));
  return KRIPKE_OK;
}

// Enqueue a tiered fast census: one init, then one launch per tier, each in
// its tier's mode (`mode` names the position space of p0, p1: both tiers
// share it).  The device order array must already hold t.order.
int enqueue_tiered(DeviceState* ds, const DeviceBatch& db, const Tiering& t, int n, int nvars,
                   int mode, bool fused, uint32_t nformulas, uint64_t p0, uint64_t p1,
                   unsigned long long* key, unsigned long long* cnt, bool decide,
                   unsigned long long* queues, hipStream_t s, int ipw, uint32_t out_stride = 2,
                   const uint32_t* list_succ = nullptr, uint32_t* valid_bits = nullptr,
                   uint64_t valid_words = 0) {
  KR_HIP(launch_init(key, cnt, out_stride, fused ? 4 * nformulas : nformulas, nullptr, s));
  (void)mode;
  int rc = enqueue_fast(ds, db, n, nvars, t.ls_a, t.mode_a, fused, t.count_a, p0, p1, key, cnt,
                        decide, queues, s, ipw, 0, 0, false, nformulas, out_stride, list_succ,
                        valid_bits, valid_words);
  if (rc || t.count_a == (uint32_t)t.order.size()) return rc;
  return enqueue_fast(ds, db, n, nvars, t.ls_b, t.mode_b, fused,
                      (uint32_t)t.order.size() - t.count_a, p0, p1, key, cnt, decide, queues + 1,
                      s, ipw, 0, t.count_a, false, nformulas, out_stride, list_succ,
                      valid_bits, valid_words);
}

int upload_order(const Tiering& t, uint32_t* d_order, hipStream_t s) {
  KR_HIP(hipMemcpyAsync(d_order, t.order.data(), t.order.size() * 4, hipMemcpyHostToDevice, s));
  KR_HIP(hipStreamSynchronize(s));
  return KRIPKE_OK;
}

}  // namespace

// ------------------------------------------------- allocation-free census
// Fixed device scratch of kripke_census_range_static: the two work-queue
// counters, the program offsets, the launch order and the micro-op code of one
// batch, at the offsets below.  Every device holds its own copy until the
// process ends.  Host code never names the array in a device context: it uses
// the address hipGetSymbolAddress returns for the current device.
constexpr uint64_t kStQueue = 0;  // 2 x u64
constexpr uint64_t kStOff = 256;  // u32[max formulas + 1]
constexpr uint64_t kStOrder =
    kStOff + ((4ull * (KRIPKE_STATIC_MAX_FORMULAS + 1) + 255) & ~255ull);  // u32[max + 1]
constexpr uint64_t kStCode =
    kStOrder + ((4ull * (KRIPKE_STATIC_MAX_FORMULAS + 1) + 255) & ~255ull);
constexpr uint64_t kStBytes = kStCode + KRIPKE_STATIC_MAX_CODE;

static __device__ __align__(256) uint8_t scratch[kStBytes];

namespace {

std::map<int, uint8_t*> g_scratch;  // device ordinal -> address of its `scratch`

// Address of the current device's scratch, looked up once per device.
int static_scratch(uint8_t** out) {
  int dev = 0;
  KR_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_scratch.find(dev);
  if (it == g_scratch.end()) {
    void* p = nullptr;
    KR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(KRIPKE_EHIP, "hipGetSymbolAddress returned no address for scratch");
    it = g_scratch.emplace(dev, static_cast<uint8_t*>(p)).first;
  }
  *out = it->second;
  return KRIPKE_OK;
}

// The DeviceBatch of a compiled batch placed in the static scratch; the
// order area receives `order` (the tier order of the fast path or the batch's
// cost order).  Waits for the copies: the host vectors die with the caller.
int stage_static(uint8_t* base, const MicroBatch& mb, const std::vector<uint32_t>& order,
                 DeviceBatch* db, hipStream_t s) {
  db->queue = reinterpret_cast<unsigned long long*>(base + kStQueue);
  db->uoff = reinterpret_cast<uint32_t*>(base + kStOff);
  db->order = reinterpret_cast<uint32_t*>(base + kStOrder);
  db->ucode = base + kStCode;
  KR_HIP(hipMemcpyAsync(db->ucode, mb.code.data(), mb.code.size(), hipMemcpyHostToDevice, s));
  KR_HIP(hipMemcpyAsync(db->uoff, mb.off.data(), mb.off.size() * 4, hipMemcpyHostToDevice, s));
  KR_HIP(hipMemcpyAsync(db->order, order.data(), order.size() * 4, hipMemcpyHostToDevice, s));
  KR_HIP(hipStreamSynchronize(s));
  return KRIPKE_OK;
}

}  // namespace

static int check_range_args(uint32_t nformulas, uint32_t n, uint32_t cls, uint32_t nvars,
                     uint64_t frame_begin, uint64_t frame_end, uint32_t flags,
                     const kripke_census_result* d_out) {
  if (nformulas == 0 || !d_out) return fail(KRIPKE_EINVAL, "empty batch or null output");
  if (cls > KRIPKE_S5) return fail(KRIPKE_EINVAL, "unknown frame class");
  if (flags > KRIPKE_DECIDE) return fail(KRIPKE_EINVAL, "unknown flags");
  int rc = check_sizes(n, nvars, 6);
  if (rc) return rc;
  const uint64_t nframes = 1ull << (n * n);
  if (frame_begin > frame_end || frame_end > nframes)
    return fail(KRIPKE_EINVAL, "frame range outside [0, 2^(n*n))");
  return KRIPKE_OK;
}

// ================================================================= C ABI
extern "C" {

const char* kripke_last_error(void) { return g_err.c_str(); }

int kripke_version(void) { return 100; }

void kripke_key_decode(uint64_t key, uint32_t n, uint32_t nvars, uint64_t* frame,
                       uint64_t* valuation, uint32_t* world) {
  const uint32_t sh = nvars * n + 4;
  if (frame) *frame = sh >= 64 ? 0 : key >> sh;
  if (valuation) *valuation = (key >> 4) & ((1ull << (nvars * n)) - 1);
  if (world) *world = (uint32_t)(key & 15u);
}

void kripke_frame_decode(uint64_t frame, uint32_t n, uint32_t* succ) {
  const uint64_t full = (1ull << n) - 1;
  for (uint32_t w = 0; w < n; ++w) succ[w] = (uint32_t)((frame >> (n * w)) & full);
}

int kripke_census_range(const uint8_t* code, const uint32_t* offsets, uint32_t nformulas,
                        uint32_t n, uint32_t cls, uint32_t nvars, uint64_t frame_begin,
                        uint64_t frame_end, uint32_t flags, kripke_census_result* d_out,
                        void* stream) {
  g_err.clear();
  int rc = check_range_args(nformulas, n, cls, nvars, frame_begin, frame_end, flags, d_out);
  if (rc) return rc;
  MicroBatch mb;
  if ((rc = compile_batch(code, offsets, nformulas, nvars, (int)n, false, &mb))) return rc;
  DeviceState* ds = nullptr;
  if ((rc = device_state(&ds))) return rc;
  hipStream_t s = (hipStream_t)stream;
  auto* key = reinterpret_cast<unsigned long long*>(&d_out[0].first_key);
  auto* cnt = reinterpret_cast<unsigned long long*>(&d_out[0].fail_count);
  const bool decide = flags == KRIPKE_DECIDE;
  const int mode = cls == KRIPKE_K ? 0 : 1;
  Tiering tiers;
  DeviceBatch db;
  if (cls <= KRIPKE_T && pick_tiers(mb, (int)n, (int)nvars, mode, false, &tiers)) {
    const uint64_t p0 = mode == 0 ? frame_begin : t_rank(frame_begin, (int)n);
    const uint64_t p1 = mode == 0 ? frame_end : t_rank(frame_end, (int)n);
    if ((rc = upload(mb, &db, 2, s))) return rc;
    if ((rc = upload_order(tiers, db.order, s))) return rc;
    rc = enqueue_tiered(ds, db, tiers, (int)n, (int)nvars, mode, false, nformulas, p0, p1, key,
                        cnt, decide, db.queue, s, 16);
    int rc2 = release(&db, s);
    return rc ? rc : rc2;
  }
  Scan sc;
  if ((rc = make_scan(ds, (int)n, (int)cls, frame_begin, frame_end, &sc))) return rc;
  if ((rc = upload(mb, &db, 1, s))) return rc;
  rc = enqueue_scan(ds, db, sc, (int)n, (int)nvars, nformulas, key, cnt, 2, decide,
                    false, db.queue, s);
  int rc2 = release(&db, s);
  return rc ? rc : rc2;
}

int kripke_census_range_static(const uint8_t* code, const uint32_t* offsets,
                               uint32_t nformulas, uint32_t n, uint32_t cls, uint32_t nvars,
                               uint64_t frame_begin, uint64_t frame_end, uint32_t flags,
                               kripke_census_result* d_out, void* stream) {
  g_err.clear();
  int rc = check_range_args(nformulas, n, cls, nvars, frame_begin, frame_end, flags, d_out);
  if (rc) return rc;
  if (cls > KRIPKE_T)
    return fail(KRIPKE_EINVAL, "the static-scratch census supports classes K and T only");
  if (nformulas > KRIPKE_STATIC_MAX_FORMULAS)
    return fail(KRIPKE_ELIMIT, "the static-scratch census takes at most " +
                                   std::to_string(KRIPKE_STATIC_MAX_FORMULAS) + " formulas");
  MicroBatch mb;
  if ((rc = compile_batch(code, offsets, nformulas, nvars, (int)n, false, &mb))) return rc;
  if (mb.code.size() > KRIPKE_STATIC_MAX_CODE)
    return fail(KRIPKE_ELIMIT, "compiled batch of " + std::to_string(mb.code.size()) +
                                   " bytes exceeds the static program area of " +
                                   std::to_string(KRIPKE_STATIC_MAX_CODE) + " bytes");
  DeviceState* ds = nullptr;
  if ((rc = device_state(&ds))) return rc;
  uint8_t* base = nullptr;
  if ((rc = static_scratch(&base))) return rc;
  hipStream_t s = (hipStream_t)stream;
  auto* key = reinterpret_cast<unsigned long long*>(&d_out[0].first_key);
  auto* cnt = reinterpret_cast<unsigned long long*>(&d_out[0].fail_count);
  const bool decide = flags == KRIPKE_DECIDE;
  const int mode = cls == KRIPKE_K ? 0 : 1;
  Tiering tiers;
  DeviceBatch db;
  if (pick_tiers(mb, (int)n, (int)nvars, mode, false, &tiers)) {
    const uint64_t p0 = mode == 0 ? frame_begin : t_rank(frame_begin, (int)n);
    const uint64_t p1 = mode == 0 ? frame_end : t_rank(frame_end, (int)n);
    if ((rc = stage_static(base, mb, tiers.order, &db, s))) return rc;
    return enqueue_tiered(ds, db, tiers, (int)n, (int)nvars, mode, false, nformulas, p0, p1, key,
                          cnt, decide, db.queue, s, 16);
  }
  // K and T scans need no class list, so make_scan allocates nothing here
  Scan sc;
  if ((rc = make_scan(ds, (int)n, (int)cls, frame_begin, frame_end, &sc))) return rc;
  if ((rc = stage_static(base, mb, mb.order, &db, s))) return rc;
  return enqueue_scan(ds, db, sc, (int)n, (int)nvars, nformulas, key, cnt, 2, decide, false,
                      db.queue, s);
}

int kripke_frame_validity(const uint8_t* code, const uint32_t* offsets, uint32_t nformulas,
                          uint32_t n, uint32_t nvars, uint32_t* d_bits, void* stream) {
  g_err.clear();
  if (nformulas == 0 || !d_bits) return fail(KRIPKE_EINVAL, "empty batch or null output");
  int rc = check_sizes(n, nvars, 5);
  if (rc) return rc;
  const int B0 = fast_block_log2((int)n, (int)nvars, 0, 0);
  if (n < 4 || n * nvars > 11 || B0 > 5)
    return fail(KRIPKE_ELIMIT, "frame validity maps need 4 <= n <= 5 and n * nvars <= 11");
  MicroBatch mb;
  if ((rc = compile_batch(code, offsets, nformulas, nvars, (int)n, false, &mb))) return rc;
  Tiering tiers;
  if (!pick_tiers(mb, (int)n, (int)nvars, 0, false, &tiers))
    return fail(KRIPKE_ELIMIT, "no census kernel variant for this n and nvars");
  for (int ls : {tiers.ls_a, tiers.ls_b})
    if (ls >= 0 && fast_block_log2((int)n, (int)nvars, ls, 0) > 5)
      return fail(KRIPKE_ELIMIT, "census kernel blocks wider than one bitmap word");
  DeviceState* ds = nullptr;
  if ((rc = device_state(&ds))) return rc;
  hipStream_t s = (hipStream_t)stream;
  const uint64_t nframes = 1ull << (n * n);
  const uint64_t words = (nframes + 31) / 32;
  // every map starts empty; formulas that fold to TOP are valid everywhere and
  // are skipped by the kernel, so their maps start full
  std::vector<uint32_t> fill(nformulas);
  for (uint32_t i = 0; i < nformulas; ++i) fill[i] = mb.is_const[i] == 1 ? ~0u : 0u;
  uint32_t* d_fill = nullptr;
  unsigned long long* d_res = nullptr;
  KR_HIP(hipMallocAsync((void**)&d_fill, nformulas * 4ull, s));
  KR_HIP(hipMallocAsync((void**)&d_res, nformulas * 16ull, s));
  KR_HIP(hipMemcpyAsync(d_fill, fill.data(), nformulas * 4ull, hipMemcpyHostToDevice, s));
  KR_HIP(launch_fill_rows(d_bits, words, d_fill, nformulas, s));
  KR_HIP(hipStreamSynchronize(s));
  DeviceBatch db;
  if ((rc = upload(mb, &db, 2, s))) return rc;
  if ((rc = upload_order(tiers, db.order, s))) return rc;
  rc = enqueue_tiered(ds, db, tiers, (int)n, (int)nvars, 0, false, nformulas, 0, nframes, d_res,
                      d_res + 1, false, db.queue, s, 16, 2, nullptr, d_bits, words);
  int rc2 = release(&db, s);
  KR_HIP(hipFreeAsync(d_fill, s));
  KR_HIP(hipFreeAsync(d_res, s));
  return rc ? rc : rc2;
}

int kripke_census(const uint8_t* code, const uint32_t* offsets, uint32_t nformulas, uint32_t n,
                  uint32_t cls, uint32_t nvars, kripke_census_result* d_out, void* stream) {
  g_err.clear();
  if (n < 1 || n > 5) return fail(KRIPKE_ELIMIT, "kripke_census supports 1 <= n <= 5");
  return kripke_census_range(code, offsets, nformulas, n, cls, nvars, 0, 1ull << (n * n),
                             KRIPKE_COUNT, d_out, stream);
}

int kripke_split_batch(const uint8_t* code, const uint32_t* offsets, uint32_t npairs,
                       const uint32_t* d_frames, uint64_t nframes, uint32_t n, uint32_t nvars,
                       uint64_t* d_first_key, void* stream) {
  g_err.clear();
  if (npairs == 0 || !d_first_key || (!d_frames && nframes))
    return fail(KRIPKE_EINVAL, "empty batch or null pointer");
  if (n < 1 || n > 16) return fail(KRIPKE_ELIMIT, "split supports 1 <= n <= 16");
  if (nvars > 4 || (n >= 7 && nvars > 3) || (n >= 9 && nvars > 1 && n * nvars > 24))
    return fail(KRIPKE_ELIMIT, "split supports nvars <= 4 (<= 3 for n >= 7) and, from 9 worlds, "
                               "nvars * n <= 24");
  int posbits = 0;
  while (posbits < 64 && (1ull << posbits) < nframes) ++posbits;
  if (posbits + (int)(nvars * n) + 4 > 64) return fail(KRIPKE_ELIMIT, "key does not fit 64 bits");
  MicroBatch mb;
  int rc;
  if ((rc = compile_batch(code, offsets, npairs, nvars, (int)n, true, &mb))) return rc;
  DeviceState* ds = nullptr;
  if ((rc = device_state(&ds))) return rc;
  hipStream_t s = (hipStream_t)stream;
  DeviceBatch db;
  // frames of 11..16 worlds: world-set bitmasks per lane; KRIPKE_SPLIT_WORLDMASK=1
  // selects that kernel at any size (for comparison)
  const char* force_wm = getenv("KRIPKE_SPLIT_WORLDMASK");
  if (n > 10 || (n >= 9 && nvars >= 2) || (force_wm && atoi(force_wm))) {
    if (nvars * n > 24) return fail(KRIPKE_ELIMIT, "world-mask split needs nvars * n <= 24");
    if ((rc = upload(mb, &db, 1, s))) return rc;
    WorldMaskArgs a{};
    a.ucode = db.ucode;
    a.uoff = db.uoff;
    a.order = db.order;
    a.frames = d_frames;
    a.nframes = nframes;
    a.n = n;
    a.nvars = nvars;
    const uint64_t units = nframes << (nvars * n);
    const uint64_t nblocks = (units + 63) / 64;
    const uint64_t waves = (uint64_t)ds->cus * 16;
    uint64_t bpi = std::max<uint64_t>(1, (nblocks * npairs + 16 * waves - 1) / (16 * waves));
    bpi = std::min<uint64_t>(bpi, 1ull << 16);
    a.blocks_per_item = bpi;
    a.items_per_pair = (nblocks + bpi - 1) / bpi;
    a.total_items = a.items_per_pair * npairs;
    a.queue = db.queue;
    a.out_key = reinterpret_cast<unsigned long long*>(d_first_key);
    rc = KRIPKE_OK;
    hipError_t e = launch_init(a.out_key, nullptr, 1, npairs, db.queue, s);
    if (e == hipSuccess && a.total_items) {
      const uint64_t grid = std::min<uint64_t>((uint64_t)ds->cus * 4, (a.total_items + 3) / 4);
      e = launch_split_worldmask(a, (int)std::max<uint64_t>(grid, 1), s);
    }
    if (e != hipSuccess) rc = fail(KRIPKE_EHIP, std::string("world-mask split: ") + hipGetErrorString(e));
    int rc2 = release(&db, s);
    return rc ? rc : rc2;
  }
  // wave-uniform list frames when the lanes can hold valuations only;
  // KRIPKE_SPLIT_GENERIC=1 forces the per-lane-frame kernel (for comparison)
  // (two list frames per block where a frame's valuations fill only two sets
  // of a wave; KRIPKE_SPLIT_ONE_FRAME=1 keeps one frame per block)
  const char* force_generic = getenv("KRIPKE_SPLIT_GENERIC");
  const char* one_frame = getenv("KRIPKE_SPLIT_ONE_FRAME");
  Tiering tiers;
  if (!(force_generic && atoi(force_generic)) &&
      ((!(one_frame && atoi(one_frame)) && pick_tiers(mb, (int)n, (int)nvars, 3, false, &tiers)) ||
       pick_tiers(mb, (int)n, (int)nvars, 2, false, &tiers))) {
    if ((rc = upload(mb, &db, 2, s))) return rc;
    if ((rc = upload_order(tiers, db.order, s))) return rc;
    rc = enqueue_tiered(ds, db, tiers, (int)n, (int)nvars, 2, false, npairs, 0, nframes,
                        reinterpret_cast<unsigned long long*>(d_first_key), nullptr, true,
                        db.queue, s, 16, 1, d_frames);
    int rc2 = release(&db, s);
    return rc ? rc : rc2;
  }
  Scan sc;
  sc.mode = M_LIST_SUCC;
  sc.list_succ = d_frames;
  sc.pos_begin = 0;
  sc.npos = nframes;
  if ((rc = upload(mb, &db, 1, s))) return rc;
  rc = enqueue_scan(ds, db, sc, (int)n, (int)nvars, npairs,
                    reinterpret_cast<unsigned long long*>(d_first_key), nullptr, 1, true, true,
                    db.queue, s);
  int rc2 = release(&db, s);
  return rc ? rc : rc2;
}

int kripke_split(const uint8_t* phi, uint32_t len_phi, const uint8_t* psi, uint32_t len_psi,
                 const uint32_t* d_frames, uint64_t nframes, uint32_t n, uint32_t nvars,
                 uint64_t* d_first_key, void* stream) {
  g_err.clear();
  if (!phi || !psi) return fail(KRIPKE_EINVAL, "null program");
  std::vector<uint8_t> code(phi, phi + len_phi);
  code.insert(code.end(), psi, psi + len_psi);
  uint32_t off[3] = {0, len_phi, len_phi + len_psi};
  return kripke_split_batch(code.data(), off, 1, d_frames, nframes, n, nvars, d_first_key, stream);
}

// ---------------------------------------------------------------- plans
struct KripkePlan {
  int n = 0, nvars = 0;
  uint32_t nformulas = 0, class_mask = 0;
  MicroBatch mb;
  DeviceBatch db;
  Scan scans[4];
  DeviceState* ds = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  kripke_census_result* graph_out = nullptr;
  int ls = -1;   // frame sets per lane (log2) of the fused launch, -1 = none
  int ipw = 16;  // work items per wave
  Tiering tiers;
  bool plain = false;  // one launch per formula, no graph
};

static int plan_enqueue(KripkePlan* p, kripke_census_result* d_out, hipStream_t s,
                        uint64_t frames);
static void plan_free(KripkePlan* p);

// The unbatched baselines, one launch (pair) per formula, each restricted to
// that formula through a one-entry slice of the order array:
//   - plain (p->ls < 0): per class, an (init, census) pair per formula with
//     the default tiles;
//   - per-formula + autotuned (p->ls >= 0): the fused all-class kernel with
//     the tuned tiles, one launch per formula, over frames [0, frames) (0 =
//     all), so only batching separates it from the batched plan.
static int plan_enqueue_plain(KripkePlan* p, kripke_census_result* d_out, hipStream_t s,
                              uint64_t frames = 0, uint32_t count = 0) {
  if (p->ls >= 0) {
    // count: launch only formulas 0 .. count-1 of the batch (0 = all); the autotuner
    // times candidates on such a subset, the same one whatever the candidate's tiers
    const uint64_t nf = frames ? frames : 1ull << (p->n * p->n);
    auto* key = reinterpret_cast<unsigned long long*>(&d_out[0].first_key);
    auto* cnt = reinterpret_cast<unsigned long long*>(&d_out[0].fail_count);
    KR_HIP(launch_init(key, cnt, 2, 4 * p->nformulas, nullptr, s));
    for (uint32_t i = 0; i < p->nformulas; ++i) {
      if (count && p->tiers.order[i] >= count) continue;
      const int ls = i < p->tiers.count_a ? p->tiers.ls_a : p->tiers.ls_b;
      int rc = enqueue_fast(p->ds, p->db, p->n, p->nvars, ls, 0, true, 1, 0, nf, key, cnt, false,
                            p->db.queue, s, p->ipw, 0, i, false, p->nformulas);
      if (rc) return rc;
    }
    return KRIPKE_OK;
  }
  for (int c = 0; c < 4; ++c) {
    if (!((p->class_mask >> c) & 1u)) continue;
    kripke_census_result* row = d_out + (size_t)c * p->nformulas;
    const int mode = c == KRIPKE_K ? 0 : 1;
    const int ls = c <= KRIPKE_T ? pick_sets(p->n, p->nvars, mode, false, p->mb.max_slots) : -1;
    const uint64_t nf = 1ull << (p->n * p->n);
    for (uint32_t i = 0; i < p->nformulas; ++i) {
      const uint32_t f = p->mb.order[i];
      DeviceBatch one = p->db;
      one.order = p->db.order + i;
      // the kernel indexes outputs by formula id, so pass the row base and
      // let the init kernel clear only entry f
      auto* key = reinterpret_cast<unsigned long long*>(&row[0].first_key);
      auto* cnt = reinterpret_cast<unsigned long long*>(&row[0].fail_count);
      int rc;
      if (ls >= 0) {
        rc = enqueue_fast(p->ds, one, p->n, p->nvars, ls, mode, false, 1, 0,
                          mode == 0 ? nf : t_rank(nf, p->n), key, cnt, false, p->db.queue + c,
                          s, 16, f);
      } else {
        rc = enqueue_scan(p->ds, one, p->scans[c], p->n, p->nvars, 1, key, cnt, 2, false, false,
                          p->db.queue + c, s, f);
      }
      if (rc) return rc;
    }
  }
  return KRIPKE_OK;
}

// ------------------------------------------------------------ autotuner
// Tiles: frame sets per lane (2^ls, i.e. valuation words each lane carries
// per dispatch) and work items per wave (load-balance granularity of the
// persistent queue).  Every candidate is timed on a prefix slice of the
// frames; the choice is cached in a small JSON file keyed by device, shape
// and a hash of the compiled batch.
static int plan_enqueue_any(KripkePlan* p, kripke_census_result* d_out, hipStream_t s,
                            uint64_t frames, uint32_t count = 0) {
  return p->plain ? plan_enqueue_plain(p, d_out, s, frames, count)
                  : plan_enqueue(p, d_out, s, frames);
}

static std::string tune_key(const KripkePlan* p) {
  uint64_t h = 1469598103934665603ull;
  for (uint8_t b : p->mb.code) h = (h ^ b) * 1099511628211ull;
  hipDeviceProp_t prop;
  int dev = 0;
  char arch[sizeof prop.gcnArchName] = "unknown-device";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
  char buf[256];
  snprintf(buf, sizeof buf, "%s/%dcu/n%d/v%d/m%u/B%u/h%016llx%s", arch, p->ds->cus,
           p->n, p->nvars, p->class_mask, p->nformulas, (unsigned long long)h,
           p->plain ? "/per-formula" : "");
  for (char* c = buf; *c; ++c)
    if (*c == '"' || *c == '\\') *c = '_';
  return buf;
}

static bool tune_lookup(const char* path, const std::string& key, int* ls, int* ipw) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool hit = false;
  while (fgets(line, sizeof line, f)) {
    const char* q = strstr(line, key.c_str());
    if (!q || q == line || q[-1] != '"' || q[key.size()] != '"') continue;
    const char* l = strstr(q, "\"ls\":");
    const char* w = strstr(q, "\"ipw\":");
    if (l && w) {
      *ls = atoi(l + 5);
      *ipw = atoi(w + 6);
      hit = true;
    }
  }
  fclose(f);
  return hit;
}

static void tune_store(const char* path, const std::string& key, int ls, int ipw, double ms) {
  std::vector<std::string> lines;
  if (FILE* f = fopen(path, "r")) {
    char line[512];
    while (fgets(line, sizeof line, f)) {
      std::string l(line);
      if (l.find("\"ls\":") != std::string::npos && l.find("\"" + key + "\"") == std::string::npos) {
        while (!l.empty() && (l.back() == '\n' || l.back() == ',')) l.pop_back();
        lines.push_back(l);
      }
    }
    fclose(f);
  }
  char buf[512];
  snprintf(buf, sizeof buf, "  \"%s\": {\"ls\": %d, \"ipw\": %d, \"slice_ms\": %.3f}", key.c_str(),
           ls, ipw, ms);
  lines.push_back(buf);
  std::string tmp = std::string(path) + ".tmp";
  if (FILE* f = fopen(tmp.c_str(), "w")) {
    fputs("{\n", f);
    for (size_t i = 0; i < lines.size(); ++i)
      fprintf(f, "%s%s\n", lines[i].c_str(), i + 1 < lines.size() ? "," : "");
    fputs("}\n", f);
    fclose(f);
    rename(tmp.c_str(), path);
  }
}

static int tune_plan(KripkePlan* p, const char* path) {
  const std::string key = tune_key(p);
  int ls = p->ls, ipw = p->ipw;
  Tiering t;
  if (tune_lookup(path, key, &ls, &ipw) && ipw > 0 &&
      make_tiers(p->mb, p->n, p->nvars, 0, true, ls, &t)) {
    p->ls = ls;
    p->ipw = ipw;
    p->tiers = t;
    return upload_order(t, p->db.order, p->cap);
  }
  // trial outputs and timing events, released on every return path
  struct Trial {
    kripke_census_result* out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Trial() {
      if (out) (void)hipFree(out);
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } trial;
  KR_HIP(hipMalloc(&trial.out, sizeof(kripke_census_result) * 4 * p->nformulas));
  KR_HIP(hipEventCreate(&trial.e0));
  KR_HIP(hipEventCreate(&trial.e1));
  kripke_census_result* trial_out = trial.out;
  hipEvent_t e0 = trial.e0, e1 = trial.e1;
  const uint64_t slice = std::min<uint64_t>(1ull << (p->n * p->n), 1ull << 20);
  // the per-formula form is timed on the batch's first 256 formulas (its cost is one
  // launch per formula, so the whole batch would cost 24 x nformulas launches)
  const uint32_t count = p->plain ? std::min<uint32_t>(p->nformulas, 256) : 0;
  const bool verbose = getenv("KRIPKE_TUNE_LOG") && atoi(getenv("KRIPKE_TUNE_LOG"));
  double best = 1e300;
  int best_ls = p->ls, best_ipw = p->ipw;
  // every candidate computes the same slice; its results must be identical
  std::vector<kripke_census_result> first_res, res(4 * (size_t)p->nformulas);
  for (int l = 0; l <= 3; ++l) {
    if (!make_tiers(p->mb, p->n, p->nvars, 0, true, l, &t)) continue;
    p->tiers = t;
    int rc0 = upload_order(t, p->db.order, p->cap);
    if (rc0) return rc0;
    for (int w : {4, 16, 64}) {
      p->ls = l;
      p->ipw = w;
      int rc = plan_enqueue_any(p, trial_out, p->cap, slice, count);  // warm
      if (rc) return rc;
      KR_HIP(hipEventRecord(e0, p->cap));
      if ((rc = plan_enqueue_any(p, trial_out, p->cap, slice, count))) return rc;
      KR_HIP(hipEventRecord(e1, p->cap));
      KR_HIP(hipEventSynchronize(e1));
      float ms = 0;
      KR_HIP(hipEventElapsedTime(&ms, e0, e1));
      KR_HIP(hipMemcpy(res.data(), trial_out, res.size() * sizeof(res[0]), hipMemcpyDeviceToHost));
      if (first_res.empty()) {
        first_res = res;
      } else if (memcmp(first_res.data(), res.data(), res.size() * sizeof(res[0])) != 0) {
        return fail(KRIPKE_EINTERNAL, "autotuner: tile candidate ls=" + std::to_string(l) +
                                          " ipw=" + std::to_string(w) +
                                          " disagrees with the first candidate");
      }
      if (verbose)
        fprintf(stderr, "[kripke tune] %s ls=%d ipw=%d: %.3f ms on %llu frames\n",
                p->plain ? "per-formula" : "batched", l, w, ms, (unsigned long long)slice);
      if (ms < best) {
        best = ms;
        best_ls = l;
        best_ipw = w;
      }
    }
  }
  p->ls = best_ls;
  p->ipw = best_ipw;
  make_tiers(p->mb, p->n, p->nvars, 0, true, best_ls, &p->tiers);
  if (int rc1 = upload_order(p->tiers, p->db.order, p->cap)) return rc1;
  tune_store(path, key, best_ls, best_ipw, best);
  return KRIPKE_OK;
}

int kripke_program_stats(const uint8_t* code, const uint32_t* offsets, uint32_t nformulas,
                         uint32_t nvars, int32_t* stats) {
  g_err.clear();
  if (!code || !offsets || !stats) return fail(KRIPKE_EINVAL, "null pointer");
  if (nvars > 4) return fail(KRIPKE_ELIMIT, "nvars must be <= 4");
  for (uint32_t i = 0; i < nformulas; ++i) {
    if (offsets[i + 1] < offsets[i]) return fail(KRIPKE_EINVAL, "offsets must be non-decreasing");
    Compiled c;
    std::string err;
    int rc = compile_program(code + offsets[i], offsets[i + 1] - offsets[i], nvars, &c, &err);
    if (rc) return fail(rc, "formula " + std::to_string(i) + ": " + err);
    int32_t* o = stats + 6 * (size_t)i;
    o[0] = c.modal;
    o[1] = c.binary;
    o[2] = c.loads;
    o[3] = c.saves;
    o[4] = c.slots;
    o[5] = c.is_const;
  }
  return KRIPKE_OK;
}

int kripke_signatures(const uint8_t* code, const uint32_t* offsets, uint32_t nformulas,
                      uint32_t nvars, const uint64_t* samples, uint32_t nsamples, uint64_t* d_sig,
                      void* stream) {
  g_err.clear();
  if (!samples || !d_sig || nformulas == 0) return fail(KRIPKE_EINVAL, "null pointer or empty batch");
  if (nsamples == 0 || nsamples % 64) return fail(KRIPKE_EINVAL, "nsamples must be a multiple of 64");
  if (nvars > 4) return fail(KRIPKE_ELIMIT, "nvars must be <= 4");
  const uint32_t ngroups = nsamples / 64;
  std::vector<uint32_t> groups[4];
  for (uint32_t g = 0; g < ngroups; ++g) {
    const uint32_t n = (uint32_t)(samples[g * 64ull] >> 60);
    for (uint32_t l = 0; l < 64; ++l) {
      const uint64_t smp = samples[g * 64ull + l];
      const uint32_t sn = (uint32_t)(smp >> 60);
      const uint64_t f = (smp >> 24) & 0xFFFFFFFFFull;
      const uint64_t val = (smp >> 4) & 0xFFFFFu;
      if (sn != n || n < 1 || n > 3 || f >= (1ull << (n * n)) || val >= (1ull << (nvars * n)) ||
          (smp & 15u) >= n)
        return fail(KRIPKE_EINVAL, "sample " + std::to_string(g * 64 + l) + " is invalid or "
                                   "its group of 64 mixes world counts");
    }
    groups[n].push_back(g);
  }
  MicroBatch mb;
  int rc;
  if ((rc = compile_batch(code, offsets, nformulas, nvars, 3, false, &mb))) return rc;
  hipStream_t s = (hipStream_t)stream;
  DeviceBatch db;
  if ((rc = upload(mb, &db, 1, s))) return rc;
  uint64_t* d_samples = nullptr;
  uint32_t* d_groups = nullptr;
  KR_HIP(hipMallocAsync((void**)&d_samples, nsamples * 8ull, s));
  KR_HIP(hipMallocAsync((void**)&d_groups, ngroups * 4ull, s));
  KR_HIP(hipMemcpyAsync(d_samples, samples, nsamples * 8ull, hipMemcpyHostToDevice, s));
  std::vector<uint32_t> all;
  for (int n = 1; n <= 3; ++n) all.insert(all.end(), groups[n].begin(), groups[n].end());
  KR_HIP(hipMemcpyAsync(d_groups, all.data(), all.size() * 4, hipMemcpyHostToDevice, s));
  KR_HIP(hipStreamSynchronize(s));
  uint32_t at = 0;
  for (int n = 1; n <= 3; ++n) {
    if (groups[n].empty()) continue;
    SigArgs a{};
    a.ucode = db.ucode;
    a.uoff = db.uoff;
    a.nformulas = nformulas;
    a.samples = d_samples;
    a.groups = d_groups + at;
    a.ngroups = (uint32_t)groups[n].size();
    a.words = ngroups;
    a.sig = reinterpret_cast<unsigned long long*>(d_sig);
    KR_HIP(launch_signatures(a, n, (int)nvars, s));
    at += a.ngroups;
  }
  KR_HIP(hipFreeAsync(d_samples, s));
  KR_HIP(hipFreeAsync(d_groups, s));
  return release(&db, s);
}

int kripke_knn_pairs(const uint64_t* d_sig, uint32_t nformulas, uint32_t words, uint32_t k,
                     uint64_t* d_pairs, uint64_t* d_npairs, void* stream) {
  g_err.clear();
  if (!d_sig || !d_pairs || !d_npairs) return fail(KRIPKE_EINVAL, "null pointer");
  if (nformulas > 16384 || words == 0 || words * 64 > 8192 || k == 0 || k >= nformulas)
    return fail(KRIPKE_ELIMIT, "need nformulas <= 16384, 0 < words*64 <= 8192, 0 < k < nformulas");
  hipStream_t s = (hipStream_t)stream;
  uint32_t* nbr = nullptr;
  KR_HIP(hipMallocAsync((void**)&nbr, (uint64_t)nformulas * k * 4, s));
  KR_HIP(launch_knn(d_sig, nformulas, words, k, nbr, s));
  int rc = knn_pairs_canonical(nbr, nformulas, k, d_pairs, d_npairs, s);
  if (rc) return fail(rc, "pair sort failed");
  KR_HIP(hipFreeAsync(nbr, s));
  return KRIPKE_OK;
}

int kripke_pair_hamming(const uint64_t* d_sig, uint32_t words, const uint64_t* d_pairs,
                        uint64_t npairs, uint32_t* d_dist, void* stream) {
  g_err.clear();
  if (!d_sig || (!d_pairs && npairs) || (!d_dist && npairs)) return fail(KRIPKE_EINVAL, "null pointer");
  KR_HIP(launch_pair_hamming(d_sig, words, d_pairs, npairs, d_dist, (hipStream_t)stream));
  return KRIPKE_OK;
}

int kripke_select_top(const float* d_scores, uint64_t n, uint64_t budget, uint64_t* d_idx,
                      void* stream) {
  g_err.clear();
  if (!d_scores || !d_idx || n == 0) return fail(KRIPKE_EINVAL, "null pointer or empty input");
  if (n > 0x7FFFFFFFull) return fail(KRIPKE_ELIMIT, "at most 2^31 - 1 scores");
  int rc = select_top(d_scores, n, budget, d_idx, (hipStream_t)stream);
  if (rc) return fail(rc, "score sort failed");
  return KRIPKE_OK;
}

// ---------------------------------------------------------------- MLP
int kripke_mlp_create(uint64_t seed, uint32_t max_batch, void** mlp) {
  g_err.clear();
  if (!mlp || max_batch == 0 || max_batch % 64 || max_batch > (1u << 20))
    return fail(KRIPKE_EINVAL, "max_batch must be a positive multiple of 64 (<= 2^20)");
  auto* S = new MlpState();
  S->max_batch = max_batch;
  const uint64_t B = max_batch;
  struct A { void** p; uint64_t bytes; } allocs[] = {
      {(void**)&S->params, kParams * 4}, {(void**)&S->grads, kParams * 4},
      {(void**)&S->m1, kParams * 4},     {(void**)&S->m2, kParams * 4},
      {(void**)&S->w1b, (uint64_t)kH1 * kIn * 2}, {(void**)&S->w2b, (uint64_t)kH2 * kH1 * 2},
      {(void**)&S->w2tb, (uint64_t)kH2 * kH1 * 2}, {(void**)&S->a1, B * kH1 * 2},
      {(void**)&S->a1t, B * kH1 * 2},    {(void**)&S->a2b, B * kH2 * 2},
      {(void**)&S->a2, B * kH2 * 4},     {(void**)&S->logit, B * 4},
      {(void**)&S->dz, B * 4},           {(void**)&S->lossv, B * 4},
      {(void**)&S->dh2f, B * kH2 * 4},   {(void**)&S->dh1f, B * kH1 * 4},
      {(void**)&S->dh2, B * kH2 * 2},    {(void**)&S->dh2t, B * kH2 * 2},
      {(void**)&S->dh1t, B * kH1 * 2}};
  for (auto& a : allocs)
    if (hipMalloc(a.p, a.bytes) != hipSuccess) {
      kripke_mlp_destroy(S);
      return fail(KRIPKE_ENOMEM, "device allocation failed");
    }
  // He initialisation, N(0, 2 / fan_in), Box-Muller on SplitMix64 uniforms; biases 0.
  std::vector<float> p(kParams, 0.f);
  uint64_t st = seed;
  auto next = [&]() {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  auto gauss = [&]() {
    const double u1 = ((next() >> 11) + 1.0) / 9007199254740993.0;
    const double u2 = (next() >> 11) / 9007199254740992.0;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  };
  for (uint64_t i = 0; i < (uint64_t)kH1 * kIn; ++i) p[kOffW1 + i] = (float)(gauss() * sqrt(2.0 / kIn));
  for (uint64_t i = 0; i < (uint64_t)kH2 * kH1; ++i) p[kOffW2 + i] = (float)(gauss() * sqrt(2.0 / kH1));
  for (uint64_t i = 0; i < kH2; ++i) p[kOffW3 + i] = (float)(gauss() * sqrt(2.0 / kH2));
  *mlp = S;
  return kripke_mlp_set_params(S, p.data());
}

int kripke_mlp_destroy(void* mlp) {
  auto* S = static_cast<MlpState*>(mlp);
  if (!S) return KRIPKE_OK;
  void* ptrs[] = {S->params, S->grads, S->m1, S->m2, S->w1b, S->w2b, S->w2tb, S->a1, S->a1t,
                  S->a2b, S->a2, S->logit, S->dz, S->lossv, S->dh2f, S->dh1f, S->dh2, S->dh2t,
                  S->dh1t};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete S;
  return KRIPKE_OK;
}

int kripke_mlp_set_params(void* mlp, const float* params) {
  g_err.clear();
  auto* S = static_cast<MlpState*>(mlp);
  if (!S || !params) return fail(KRIPKE_EINVAL, "null pointer");
  KR_HIP(hipMemcpy(S->params, params, kParams * 4, hipMemcpyHostToDevice));
  KR_HIP(hipMemset(S->m1, 0, kParams * 4));
  KR_HIP(hipMemset(S->m2, 0, kParams * 4));
  KR_HIP(hipMemset(S->grads, 0, kParams * 4));
  S->step = 0;
  KR_HIP(mlp_refresh(*S, nullptr));
  KR_HIP(hipDeviceSynchronize());
  return KRIPKE_OK;
}

int kripke_mlp_get_params(void* mlp, float* params) {
  g_err.clear();
  auto* S = static_cast<MlpState*>(mlp);
  if (!S || !params) return fail(KRIPKE_EINVAL, "null pointer");
  KR_HIP(hipDeviceSynchronize());
  KR_HIP(hipMemcpy(params, S->params, kParams * 4, hipMemcpyDeviceToHost));
  return KRIPKE_OK;
}

int kripke_mlp_get_grads(void* mlp, float* grads) {
  g_err.clear();
  auto* S = static_cast<MlpState*>(mlp);
  if (!S || !grads) return fail(KRIPKE_EINVAL, "null pointer");
  KR_HIP(hipDeviceSynchronize());
  KR_HIP(hipMemcpy(grads, S->grads, kParams * 4, hipMemcpyDeviceToHost));
  return KRIPKE_OK;
}

int kripke_mlp_forward(void* mlp, const uint64_t* d_sig, uint32_t words, const uint64_t* d_pairs,
                       uint64_t npairs, float* d_logits, void* stream) {
  g_err.clear();
  auto* S = static_cast<MlpState*>(mlp);
  if (!S || !d_sig || (npairs && (!d_pairs || !d_logits))) return fail(KRIPKE_EINVAL, "null pointer");
  if (words != kSigWords) return fail(KRIPKE_ELIMIT, "signatures must have 64 words (4,096 bits)");
  hipStream_t s = (hipStream_t)stream;
  for (uint64_t at = 0; at < npairs; at += S->max_batch) {
    const uint32_t m = (uint32_t)std::min<uint64_t>(S->max_batch, npairs - at);
    KR_HIP(mlp_forward(*S, d_sig, d_pairs + at, m, d_logits + at, false, s));
  }
  return KRIPKE_OK;
}

int kripke_mlp_gradients(void* mlp, const uint64_t* d_sig, uint32_t words, const uint64_t* d_pairs,
                         const float* d_labels, uint32_t m, float pos_weight, float* d_loss,
                         void* stream) {
  g_err.clear();
  auto* S = static_cast<MlpState*>(mlp);
  if (!S || !d_sig || !d_pairs || !d_labels || !d_loss) return fail(KRIPKE_EINVAL, "null pointer");
  if (words != kSigWords) return fail(KRIPKE_ELIMIT, "signatures must have 64 words (4,096 bits)");
  if (m == 0 || m % 64 || m > S->max_batch)
    return fail(KRIPKE_EINVAL, "batch must be a positive multiple of 64, <= max_batch");
  KR_HIP(mlp_backward(*S, d_sig, d_pairs, d_labels, m, pos_weight, d_loss, (hipStream_t)stream));
  return KRIPKE_OK;
}

int kripke_mlp_adam_step(void* mlp, float lr, float beta1, float beta2, float eps, void* stream) {
  g_err.clear();
  auto* S = static_cast<MlpState*>(mlp);
  if (!S) return fail(KRIPKE_EINVAL, "null handle");
  KR_HIP(mlp_adam(*S, lr, beta1, beta2, eps, (hipStream_t)stream));
  return KRIPKE_OK;
}

int kripke_calibrate_int32(double* lane_ops_per_s, void* stream) {
  g_err.clear();
  if (!lane_ops_per_s) return fail(KRIPKE_EINVAL, "null output");
  DeviceState* ds = nullptr;
  int rc = device_state(&ds);
  if (rc) return rc;
  KR_HIP(run_calibration(ds->cus, 1u << 14, lane_ops_per_s, (hipStream_t)stream));
  return KRIPKE_OK;
}

int kripke_plan_create(const uint8_t* code, const uint32_t* offsets, uint32_t nformulas,
                       uint32_t n, uint32_t class_mask, uint32_t nvars, const char* tune_cache,
                       void** plan) {
  (void)tune_cache;
  g_err.clear();
  if (!plan || nformulas == 0) return fail(KRIPKE_EINVAL, "null plan or empty batch");
  const bool plain = (class_mask & KRIPKE_PLAN_PLAIN) != 0;
  class_mask &= 0xFu;
  if (class_mask == 0) return fail(KRIPKE_EINVAL, "class_mask must select a class");
  int rc = check_sizes(n, nvars, 5);
  if (rc) return rc;
  auto* p = new KripkePlan();
  p->n = (int)n;
  p->nvars = (int)nvars;
  p->nformulas = nformulas;
  p->class_mask = class_mask;
  p->plain = plain;
  if ((rc = compile_batch(code, offsets, nformulas, nvars, (int)n, false, &p->mb)) ||
      (rc = device_state(&p->ds))) {
    delete p;
    return rc;
  }
  for (int c = 0; c < 4; ++c)
    if ((class_mask >> c) & 1u)
      if ((rc = make_scan(p->ds, (int)n, c, 0, 1ull << (n * n), &p->scans[c]))) {
        delete p;
        return rc;
      }
  // tables used inside the captured graph must exist before capture; the
  // per-formula baseline uses the fused kernel only when it is autotuned
  if (class_mask == 0xF && n <= 5 && (!plain || tune_cache) &&
      pick_tiers(p->mb, (int)n, (int)nvars, 0, true, &p->tiers))
    p->ls = p->tiers.ls_a;
  if (p->ls >= 0) {
    const uint32_t* lv = nullptr;
    if ((rc = level_table(p->ds, (int)n, &lv))) {
      delete p;
      return rc;
    }
  }
  hipError_t e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete p;
    return fail(KRIPKE_EHIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
  }
  if ((rc = upload(p->mb, &p->db, 4, p->cap)) ||
      (p->ls >= 0 && (rc = upload_order(p->tiers, p->db.order, p->cap)))) {
    (void)hipStreamDestroy(p->cap);
    delete p;
    return rc;
  }
  if (tune_cache && p->ls >= 0 && !getenv("KRIPKE_SETS_LOG2") &&
      (rc = tune_plan(p, tune_cache))) {
    const std::string msg = g_err;  // freeing the plan must not clear the message
    plan_free(p);
    g_err = msg;
    return rc;
  }
  *plan = p;
  return KRIPKE_OK;
}

static int plan_enqueue(KripkePlan* p, kripke_census_result* d_out, hipStream_t s,
                        uint64_t frames) {
  const uint64_t nf = frames ? frames : 1ull << (p->n * p->n);
  if (p->ls >= 0)  // one pass: every K frame reduces into each class containing it
    return enqueue_tiered(p->ds, p->db, p->tiers, p->n, p->nvars, 0, true, p->nformulas, 0, nf,
                          reinterpret_cast<unsigned long long*>(&d_out[0].first_key),
                          reinterpret_cast<unsigned long long*>(&d_out[0].fail_count), false,
                          p->db.queue, s, p->ipw);
  for (int c = 0; c < 4; ++c) {
    if (!((p->class_mask >> c) & 1u)) continue;
    kripke_census_result* row = d_out + (size_t)c * p->nformulas;
    const int mode = c == KRIPKE_K ? 0 : 1;
    const int ls = c <= KRIPKE_T ? pick_sets(p->n, p->nvars, mode, false, p->mb.max_slots) : -1;
    if (ls >= 0) {
      const uint64_t nf = 1ull << (p->n * p->n);
      int rc = enqueue_fast(p->ds, p->db, p->n, p->nvars, ls, mode, false, p->nformulas, 0,
                            mode == 0 ? nf : t_rank(nf, p->n),
                            reinterpret_cast<unsigned long long*>(&row[0].first_key),
                            reinterpret_cast<unsigned long long*>(&row[0].fail_count), false,
                            p->db.queue + c, s);
      if (rc) return rc;
      continue;
    }
    int rc = enqueue_scan(p->ds, p->db, p->scans[c], p->n, p->nvars, p->nformulas,
                          reinterpret_cast<unsigned long long*>(&row[0].first_key),
                          reinterpret_cast<unsigned long long*>(&row[0].fail_count), 2, false,
                          false, p->db.queue + c, s);
    if (rc) return rc;
  }
  return KRIPKE_OK;
}

int kripke_plan_launch(void* plan, kripke_census_result* d_out, void* stream) {
  g_err.clear();
  auto* p = static_cast<KripkePlan*>(plan);
  if (!p || !d_out) return fail(KRIPKE_EINVAL, "null plan or output");
  if (p->plain) return plan_enqueue_plain(p, d_out, (hipStream_t)stream);
  if (!p->exec || p->graph_out != d_out) {
    if (p->exec) {
      KR_HIP(hipGraphExecDestroy(p->exec));
      KR_HIP(hipGraphDestroy(p->graph));
      p->exec = nullptr;
    }
    KR_HIP(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    int rc = plan_enqueue(p, d_out, p->cap, 0);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap, &g);
    if (rc) return rc;
    if (e != hipSuccess) return fail(KRIPKE_EHIP, std::string("capture: ") + hipGetErrorString(e));
    p->graph = g;
    KR_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    p->graph_out = d_out;
  }
  KR_HIP(hipGraphLaunch(p->exec, (hipStream_t)stream));
  return KRIPKE_OK;
}

static void plan_free(KripkePlan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap) {
    release(&p->db, p->cap);
    (void)hipStreamSynchronize(p->cap);
    (void)hipStreamDestroy(p->cap);
  }
  delete p;
}

int kripke_plan_destroy(void* plan) {
  g_err.clear();
  if (plan) plan_free(static_cast<KripkePlan*>(plan));
  return KRIPKE_OK;
}

}  // extern "C"
