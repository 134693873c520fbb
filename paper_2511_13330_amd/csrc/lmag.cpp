// Host side of the C ABI declared in include/lmag.h: context, validation,
// system set-up, work planning, workspace and kernel sequencing.
#include "../../include/lmag.h"
#include "../../include/lmag_debug.h"
#include "internal.hpp"
#include "big.hpp"
#include "tile.hpp"
#include "pade.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace lmag;

namespace {

constexpr int TILE = 64 * 64;
constexpr int SLOT = 64 * PITCH;

struct Status {
  lmag_status code;
  std::string msg;
};

// Pade coefficients from the closed form b_j = (2m-j)! m! / ((2m)! j! (m-j)!).
void pade_coeffs(int m, double* b) {
  auto fact = [](int k) { double f = 1.0; for (int i = 2; i <= k; ++i) f *= i; return f; };
  for (int j = 0; j <= m; ++j)
    b[j] = fact(2 * m - j) * fact(m) / (fact(2 * m) * fact(j) * fact(m - j));
}

const double kTheta32_2 = 8.093024022188482e-2, kTheta32_3 = 4.258730016922831e-1;
const double kTheta64[3] = {1.495585217958292e-2, 2.539398330063230e-1, 9.504178996162932e-1};

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

struct lmag_ctx {
  int device = 0;
  int n_cu = 0;
  std::string err;
  // system
  bool has_sys = false;
  int d = 0, n = 0, ns = 0, nc = 0, nj = 0, prec = 32, order = 1, hold = 0, nb = 0, chunk = 0;
  bool tiled = false;   // block-tiled path: superoperators above 64 x 64, or Magnus order 6
  long long call_total = 0;   // slices of the current compute call (tuning key)
  size_t ws_max = 0;
  double* basis64 = nullptr;
  void* basis32 = nullptr;
  void* sp_dev = nullptr;     // sparse basis tables (64 x 64 path), see build_sparse
  int32_t* tile_lists = nullptr;   // block-tiled path: nonzero basis tiles per position
  const int32_t* tile_ptr = nullptr;
  const int32_t* tile_j = nullptr;
  SparseBasis sp{};
  // logical-subspace score of the current call (0: process fidelity)
  int score_kind = 0, score_L = 0;
  double* logP_dev = nullptr;   // [64][MAX_LOGICAL] complex
  // workspace
  char* ws = nullptr;
  size_t ws_size = 0;
  char* pinned = nullptr;
  size_t pinned_size = 0;
  std::vector<char> meta_host;     // pageable plan staging of the no-allocation entry point
  char* scratch = nullptr;         // this device's copy of the static scratch array
  hipEvent_t upload_done = nullptr;
  bool upload_pending = false;
  hipStream_t last_stream = nullptr;
  // completion of the last compute call: a call on another stream waits for it
  // on the device, since every call shares the workspace
  hipEvent_t call_done = nullptr;
  bool call_pending = false;
  int8_t* last_ms = nullptr;
  int last_total_slices = 0;
  void* dbg_scratch = nullptr;
  double* mse_part = nullptr;
  PadeTable pade{};
  // stage timers
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  int64_t plan_info[5] = {0, 0, 0, 0, 0};
  bool plan_recompute = false;
  int plan_waves = 0;
  // tuning: chosen (chunk, variant) per key. 64 x 64 path: inverse variant (0 auto,
  // 1 Gauss-Jordan, 2 Neumann); block-tiled path: product kernel (BigGemmArgs::variant)
  int inv_variant = 0;
  int big_variant = -1;          // forced product kernel of the block-tiled path (-1: tuned or default)
  bool real = false;             // block-tiled path in the real Hermitian-operator basis
  std::vector<std::pair<std::string, std::pair<int, int>>> tuned;
  bool clk_on = false;
  long long* clk_dev = nullptr;

  hipEvent_t ev_get() {
    if (!ev_pool.empty()) { hipEvent_t e = ev_pool.back(); ev_pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
    return e;
  }

  lmag_status fail(lmag_status c, const std::string& m) {
    err = m;
    return c;
  }
  lmag_status hip_fail(hipError_t e, const char* where) {
    err = std::string(where) + ": " + hipGetErrorString(e);
    return LMAG_E_DEVICE;
  }
};

namespace {

struct Plan {
  std::vector<Item> items;
  std::vector<Chunk> chunks;
  std::vector<int32_t> chunk_item, slice_item;
  std::vector<int64_t> amp_off;
  std::vector<int32_t> group_first, group_items, group_global;
  int total_slices = 0, total_chunks = 0, max_slices = 0, max_chunks = 0, n_groups = 0;
  int chunk_size = 0;
  bool recompute = false;
};

struct Layout {
  size_t items, chunks, chunk_item, slice_item, amp_off, group_first, group_items, group_global,
      meta_end;
  size_t counters, alpha, gtrace, ms, nlev, F_items, st64, st, totals, pre[2], suf[2], env,
      gscratch, omega, tiles, rscratch, total;
};

// Checks every argument of a compute call on the host before anything runs.
lmag_status validate_batch(lmag_ctx* c, const lmag_batch* b, const int32_t* target_of_item,
                           int n_targets, bool writes_grad) {
  if (!b) return c->fail(LMAG_E_INVALID, "batch is NULL");
  if (b->n_items < 1) return c->fail(LMAG_E_INVALID, "n_items must be >= 1");
  if (!b->n_slices || !b->slice_offset) return c->fail(LMAG_E_INVALID, "n_slices/slice_offset NULL");
  if (!b->amps && c->nc > 0) return c->fail(LMAG_E_INVALID, "amps is NULL");
  if (!(b->dt > 0.0) || !std::isfinite(b->dt)) return c->fail(LMAG_E_INVALID, "dt must be finite and > 0");
  if (b->n_groups < 0) return c->fail(LMAG_E_INVALID, "n_groups < 0");
  if (b->n_groups > 0 && !b->group_of_item) return c->fail(LMAG_E_INVALID, "group_of_item NULL");
  long long total = 0;
  for (int i = 0; i < b->n_items; ++i) {
    if (b->n_slices[i] < 1) return c->fail(LMAG_E_INVALID, "n_slices[i] < 1");
    if (b->slice_offset[i] < 0) return c->fail(LMAG_E_INVALID, "slice_offset[i] < 0");
    total += b->n_slices[i];
  }
  if (total > (1LL << 34)) return c->fail(LMAG_E_UNSUPPORTED, "too many slices in one call");
  if (target_of_item)
    for (int i = 0; i < b->n_items; ++i)
      if (target_of_item[i] < 0 || target_of_item[i] >= n_targets)
        return c->fail(LMAG_E_INVALID, "target_of_item out of range");
  if (b->n_groups > 0) {
    std::vector<int> first(b->n_groups, -1);
    for (int i = 0; i < b->n_items; ++i) {
      const int gi = b->group_of_item[i];
      if (gi < 0 || gi >= b->n_groups) return c->fail(LMAG_E_INVALID, "group_of_item out of range");
      if (first[gi] < 0) first[gi] = i;
      else if (b->slice_offset[i] != b->slice_offset[first[gi]] || b->n_slices[i] != b->n_slices[first[gi]])
        return c->fail(LMAG_E_INVALID, "items of a group must share amplitudes and length");
    }
    for (int gi = 0; gi < b->n_groups; ++gi)
      if (first[gi] < 0) return c->fail(LMAG_E_INVALID, "empty group");
  }
  if (writes_grad) {
    // each gradient row belongs to one item (or one group): ranges of different
    // units must not overlap, else two writers would race for the same rows
    std::vector<std::pair<int64_t, int64_t>> r;
    if (b->n_groups > 0) {
      std::vector<int> first(b->n_groups, -1);
      for (int i = 0; i < b->n_items; ++i)
        if (first[b->group_of_item[i]] < 0) {
          first[b->group_of_item[i]] = i;
          r.push_back({b->slice_offset[i], b->slice_offset[i] + b->n_slices[i]});
        }
    } else {
      for (int i = 0; i < b->n_items; ++i) r.push_back({b->slice_offset[i], b->slice_offset[i] + b->n_slices[i]});
    }
    std::sort(r.begin(), r.end());
    for (size_t k = 1; k < r.size(); ++k)
      if (r[k].first < r[k - 1].second)
        return c->fail(LMAG_E_INVALID, "amplitude rows of two items (groups) overlap in a gradient call; "
                                       "put items that share a pulse into one group");
  }
  return LMAG_OK;
}

std::string tune_key(const lmag_ctx* c, long long total) {
  int b = 0;
  while ((1LL << (b + 1)) <= total) ++b;
  // "h": the block-tiled path in the real basis of Hermitian operators
  return "p" + std::to_string(c->prec) + (c->real ? "h" : "") + "_o" + std::to_string(c->order) + "_d" +
         std::to_string(c->d) + "_s" + std::to_string(b);
}

const std::pair<int, int>* tuned_for(const lmag_ctx* c, long long total) {
  const std::string k = tune_key(c, total);
  for (auto& t : c->tuned)
    if (t.first == k) return &t.second;
  return nullptr;
}

// Automatic chunk length (slices per work unit): with up to 64 slices per
// compute unit, one chunk each; above that about four chunks per workgroup (the
// persistent kernels take chunks from a counter, which balances uneven items),
// between 64 and 256 slices. Longer chunks mean fewer chunk totals to scan and
// fewer environments (3-spin, 64 x 4096 slices: 256 measured 2 % faster than
// 64, with the same accuracy against the FP64 oracle). Recompute mode stays at
// 64: its per-workgroup scratch grows with the chunk.
int auto_chunk(const lmag_ctx* c, long long total, bool recompute) {
  if (c->chunk > 0) return c->chunk;
  // tuned choices are keyed by the whole call's size (a call split into
  // budget waves looks up the key of the call, as the autotuner stored it)
  if (const auto* t = tuned_for(c, c->call_total > 0 ? c->call_total : total)) return t->first;
  const long long per = (total + c->n_cu - 1) / std::max(1, c->n_cu);
  if (per <= 64) return (int)std::max<long long>(1, per);
  return (int)std::min<long long>(recompute ? 64 : 256, std::max<long long>(64, per / 4));
}

// Plan of one wave: the caller's items `idx` (grouped calls: whole groups,
// with wave-local group numbers).
void plan_wave(const lmag_ctx* c, const lmag_batch* b, const int32_t* target_of_item,
               const std::vector<int>& idx, Plan& p, bool recompute) {
  long long total = 0;
  for (int i : idx) total += b->n_slices[i];
  const int C = auto_chunk(c, total, recompute);
  p.chunk_size = C;
  const int n = (int)idx.size();
  p.items.resize(n);
  p.amp_off.resize(n);
  std::vector<int> gmap;
  if (b->n_groups > 0) gmap.assign(b->n_groups, -1);
  int slice = 0, chunk = 0;
  for (int li = 0; li < n; ++li) {
    const int i = idx[li];
    const int N = b->n_slices[i];
    const int L = (N + C - 1) / C;
    Item it{};
    it.first_chunk = chunk; it.n_chunks = L; it.first_slice = slice; it.n_slices = N;
    it.target = target_of_item ? target_of_item[i] : 0;
    it.src = i;
    it.group = -1;
    if (b->n_groups > 0) {
      const int g = b->group_of_item[i];
      if (gmap[g] < 0) { gmap[g] = (int)p.group_global.size(); p.group_global.push_back(g); }
      it.group = gmap[g];
    }
    p.items[li] = it;
    p.amp_off[li] = b->slice_offset[i];
    for (int k = 0; k < L; ++k) {
      Chunk ch{};
      ch.item = li; ch.first = slice + k * C; ch.count = std::min(C, N - k * C); ch.chunk = chunk + k;
      p.chunks.push_back(ch);
      p.chunk_item.push_back(li);
    }
    for (int k = 0; k < N; ++k) p.slice_item.push_back(li);
    slice += N;
    chunk += L;
    p.max_slices = std::max(p.max_slices, N);
    p.max_chunks = std::max(p.max_chunks, L);
  }
  p.total_slices = slice;
  p.total_chunks = chunk;
  // largest chunks first for the persistent kernels (all equal except item tails)
  std::stable_sort(p.chunks.begin(), p.chunks.end(),
                   [](const Chunk& a, const Chunk& b2) { return a.count > b2.count; });
  if (b->n_groups > 0) {
    p.n_groups = (int)p.group_global.size();
    std::vector<std::vector<int32_t>> g(p.n_groups);
    for (int li = 0; li < n; ++li) g[p.items[li].group].push_back(li);
    p.group_first.push_back(0);
    for (auto& v : g) {
      for (int li : v) p.group_items.push_back(li);
      p.group_first.push_back((int32_t)p.group_items.size());
    }
  }
}

Layout layout(const lmag_ctx* c, const Plan& p, int n_targets, bool grad, int grid) {
  const size_t es = (c->prec == 32 ? 8 : 16);
  const size_t tile = (size_t)TILE * es;
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
  L.items = take(p.items.size() * sizeof(Item));
  L.chunks = take(p.chunks.size() * sizeof(Chunk));
  L.chunk_item = take(p.chunk_item.size() * 4);
  L.slice_item = take(p.slice_item.size() * 4);
  L.amp_off = take(p.amp_off.size() * 8);
  L.group_first = take(p.group_first.size() * 4);
  L.group_items = take(p.group_items.size() * 4);
  L.group_global = take(p.group_global.size() * 4);
  L.meta_end = o;
  L.counters = take(256);
  L.alpha = take((size_t)p.total_slices * c->nb * 8);
  L.gtrace = grad ? take((size_t)p.total_slices * c->nb * 8) : 0;
  L.ms = take((size_t)p.total_slices * 2);
  L.nlev = take((size_t)p.total_slices);
  L.F_items = take(p.items.size() * 8);
  // target tiles, or one seed tile per item for a logical-subspace score
  const int n_st = std::max(1, c->score_kind ? std::max(n_targets, (int)p.items.size()) : n_targets);
  L.st64 = take((size_t)n_st * TILE * 16);
  L.st = take((size_t)n_st * tile);
  L.totals = take((size_t)p.total_chunks * tile);
  L.pre[0] = take((size_t)p.total_chunks * tile);
  L.pre[1] = take((size_t)p.total_chunks * tile);
  L.suf[0] = grad ? take((size_t)p.total_chunks * tile) : 0;
  L.suf[1] = grad ? take((size_t)p.total_chunks * tile) : 0;
  L.env = grad ? take((size_t)p.total_chunks * tile) : 0;
  L.gscratch = c->prec == 64 ? take((size_t)grid * 2 * SLOT * es) : 0;
  L.omega = take((size_t)p.total_slices * tile);
  L.tiles = grad && !p.recompute ? take((size_t)p.total_slices * WS_TILES * tile) : 0;
  L.rscratch = grad && p.recompute ? take((size_t)grid * p.chunk_size * WS_TILES * tile) : 0;
  L.total = o;
  return L;
}

lmag_status ensure_ws(lmag_ctx* c, size_t bytes) {
  if (c->ws_max && bytes > c->ws_max)
    return c->fail(LMAG_E_NOMEM, "workspace of " + std::to_string(bytes) +
                                     " bytes exceeds workspace_bytes_max");
  if (bytes <= c->ws_size) return LMAG_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return c->hip_fail(e, "hipDeviceSynchronize");
  if (c->ws) (void)hipFree(c->ws);
  c->ws = nullptr;
  c->ws_size = 0;
  const size_t want = align_up(bytes + bytes / 8, 1 << 20);
  e = hipMalloc((void**)&c->ws, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    c->ws = nullptr;
    return c->fail(LMAG_E_NOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
  }
  c->ws_size = want;
  return LMAG_OK;
}

lmag_status ensure_pinned(lmag_ctx* c, size_t bytes) {
  if (c->upload_pending) {
    hipError_t e = hipEventSynchronize(c->upload_done);
    if (e != hipSuccess) return c->hip_fail(e, "hipEventSynchronize");
    c->upload_pending = false;
  }
  if (bytes <= c->pinned_size) return LMAG_OK;
  if (c->pinned) (void)hipHostFree(c->pinned);
  c->pinned = nullptr;
  c->pinned_size = 0;
  const size_t want = align_up(bytes + bytes / 4, 1 << 16);
  hipError_t e = hipHostMalloc((void**)&c->pinned, want, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return c->fail(LMAG_E_NOMEM, "hipHostMalloc failed");
  }
  c->pinned_size = want;
  return LMAG_OK;
}

// Copies the plan metadata to dst (the start of the call's workspace). The host
// staging buffer is the context's pinned buffer, or with pinned = false a
// pageable host buffer of the context (the entry point that allocates no device
// or pinned memory); either is reused only after the previous upload finished.
lmag_status upload_plan(lmag_ctx* c, const Plan& p, const Layout& L, hipStream_t s, char* dst,
                        bool pinned = true) {
  char* h = nullptr;
  if (pinned) {
    lmag_status st = ensure_pinned(c, L.meta_end);
    if (st != LMAG_OK) return st;
    h = c->pinned;
  } else {
    if (c->upload_pending) {
      hipError_t e = hipEventSynchronize(c->upload_done);
      if (e != hipSuccess) return c->hip_fail(e, "hipEventSynchronize");
      c->upload_pending = false;
    }
    if (c->meta_host.size() < L.meta_end) c->meta_host.resize(L.meta_end);
    h = c->meta_host.data();
  }
  std::memset(h, 0, L.meta_end);
  auto put = [&](size_t off, const void* src, size_t bytes) { if (bytes) std::memcpy(h + off, src, bytes); };
  put(L.items, p.items.data(), p.items.size() * sizeof(Item));
  put(L.chunks, p.chunks.data(), p.chunks.size() * sizeof(Chunk));
  put(L.chunk_item, p.chunk_item.data(), p.chunk_item.size() * 4);
  put(L.slice_item, p.slice_item.data(), p.slice_item.size() * 4);
  put(L.amp_off, p.amp_off.data(), p.amp_off.size() * 8);
  put(L.group_first, p.group_first.data(), p.group_first.size() * 4);
  put(L.group_items, p.group_items.data(), p.group_items.size() * 4);
  put(L.group_global, p.group_global.data(), p.group_global.size() * 4);
  hipError_t e = hipMemcpyAsync(dst, h, L.meta_end, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return c->hip_fail(e, "hipMemcpyAsync(plan)");
  e = hipEventRecord(c->upload_done, s);
  if (e != hipSuccess) return c->hip_fail(e, "hipEventRecord");
  c->upload_pending = true;
  return LMAG_OK;
}

#define HIPCHK(expr, where)                           \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return c->hip_fail(e_, where); \
  } while (0)

// The common pipeline: alpha, forward slices, chunk scans, (environments,
// fidelity, backward slices, chain rule). Returns the index (0/1) of the final
// prefix buffer through *pre_final.
struct StageTimer {
  lmag_ctx* c;
  int stage;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  StageTimer(lmag_ctx* c_, int st, hipStream_t s_) : c(c_), stage(st), s(s_) {
    if (!c->prof) return;
    a = c->ev_get();
    b = c->ev_get();
    if (a && b) (void)hipEventRecord(a, s);
  }
  ~StageTimer() {
    if (!c->prof || !a || !b) return;
    (void)hipEventRecord(b, s);
    c->ev_pending.push_back({stage, {a, b}});
  }
};

lmag_status run(lmag_ctx* c, const lmag_batch* b, const Plan& p, const Layout& L, bool grad,
                bool fidelity, const void* U_target, int n_targets, double* F_out, void* grad_out,
                void* S_out, hipStream_t s, int grid, char* base) {
  char* w = base;
  auto at = [&](size_t off) { return (void*)(w + off); };
  const Item* items = (const Item*)at(L.items);
  const size_t es = (c->prec == 32 ? 8 : 16);
  (void)es;

  AlphaArgs aa{};
  aa.prec = c->prec; aa.amps = b->amps; aa.item_amp_offset = (const int64_t*)at(L.amp_off);
  aa.items = items; aa.n_items = (int)p.items.size(); aa.static_coef = b->static_coef;
  aa.ctrl_scale = b->ctrl_scale; aa.n_ctrl = c->nc; aa.n_static = c->ns; aa.order = c->order;
  aa.hold_foh = c->hold == LMAG_FOH; aa.nb = c->nb; aa.dt = b->dt;
  aa.slice_item = (const int32_t*)at(L.slice_item); aa.alpha = (double*)at(L.alpha);
  aa.n_slices_total = p.total_slices;
  { StageTimer t(c, 0, s); HIPCHK(launch_alpha(aa, s), "alpha"); }
  HIPCHK(launch_fill_int((int*)at(L.counters), 0, 64, s), "fill");

  SliceArgs sa{};
  sa.basis = c->prec == 32 ? c->basis32 : (const void*)c->basis64;
  sa.nb = c->nb; sa.alpha = (const double*)at(L.alpha);
  sa.chunks = (const Chunk*)at(L.chunks); sa.n_chunks = p.total_chunks;
  sa.counter = (int*)at(L.counters);
  sa.ws_tiles = grad ? at(L.tiles) : nullptr; sa.store = grad ? 1 : 0;
  sa.totals = at(L.totals); sa.env = grad ? at(L.env) : nullptr;
  sa.gtrace = grad ? (double*)at(L.gtrace) : nullptr; sa.ms = (int8_t*)at(L.ms);
  sa.nlev = (int8_t*)at(L.nlev);
  {
    int inv = c->inv_variant;
    if (inv == 0 && c->chunk <= 0)
      if (const auto* t = tuned_for(c, c->call_total > 0 ? c->call_total : p.total_slices)) inv = t->second;
    if (inv < 0 || inv > 2) inv = 0;   // a line for a block-tiled key names a product kernel
    if (inv == 1) sa.nlev = nullptr;   // Gauss-Jordan for every slice
    sa.inv_mode = inv;
  }
  sa.gscratch = c->prec == 64 ? at(L.gscratch) : nullptr; sa.pade = c->pade;
  sa.omega = at(L.omega); sa.clk = c->clk_on ? c->clk_dev : nullptr;
  sa.recompute = grad && p.recompute; sa.rscratch = sa.recompute ? at(L.rscratch) : nullptr;
  sa.max_chunk = p.chunk_size;
  sa.sp = c->sp;
  sa.real = c->real ? 1 : 0;
  if (sa.recompute) { sa.store = 0; sa.ws_tiles = nullptr; }
  { StageTimer t(c, 1, s); HIPCHK(launch_omega(c->prec, sa, p.total_slices, s), "omega"); }
  { StageTimer t(c, 2, s); HIPCHK(launch_slice_forward(c->prec, sa, grid, s), "forward"); }
  c->last_ms = (int8_t*)at(L.ms);
  c->last_total_slices = p.total_slices;

  // inclusive prefix (and suffix) of chunk totals, Hillis-Steele levels
  const bool want_suf = grad;
  const void* pre_cur = at(L.totals);
  const void* suf_cur = at(L.totals);
  int buf = 0;
  for (int st = 1; st < p.max_chunks; st <<= 1) {
    ScanArgs sc{};
    sc.prec = c->prec; sc.items = items; sc.n_items = (int)p.items.size();
    sc.n_chunks_total = p.total_chunks; sc.step = st;
    sc.pre_in = pre_cur; sc.pre_out = at(L.pre[buf]);
    sc.suf_in = want_suf ? suf_cur : nullptr; sc.suf_out = want_suf ? at(L.suf[buf]) : nullptr;
    { StageTimer t(c, 3, s); HIPCHK(launch_scan_level(sc, (const int32_t*)at(L.chunk_item), s), "scan"); }
    pre_cur = at(L.pre[buf]);
    if (want_suf) suf_cur = at(L.suf[buf]);
    buf ^= 1;
  }

  if (S_out) {
    ExtractArgs ea{};
    ea.prec = c->prec; ea.items = items; ea.n_items = (int)p.items.size(); ea.pre = pre_cur;
    ea.out = S_out; ea.n = c->n;
    HIPCHK(launch_extract(ea, s), "extract");
    if (c->real) HIPCHK(launch_out_from_real(S_out, items, ea.n_items, c->d, s), "extract (column stacking)");
  }
  if (!fidelity) return LMAG_OK;

  const bool grouped = p.n_groups > 0;
  double* F_items = grouped ? (double*)at(L.F_items) : F_out;
  if (c->score_kind) {
    // logical-subspace score: Pi, score and the per-item seed from each total
    LogicalArgs la{};
    la.prec = c->prec; la.items = items; la.n_items = (int)p.items.size(); la.pre = pre_cur;
    la.kind = c->score_kind; la.L = c->score_L; la.P = c->logP_dev; la.T = (const double*)U_target;
    la.score = F_items; la.f_by_src = grouped ? 0 : 1;
    la.st64 = (double*)at(L.st64); la.st32 = c->prec == 32 ? (float*)at(L.st) : nullptr;
    la.real = c->real ? 1 : 0;
    { StageTimer t(c, 4, s); HIPCHK(launch_logical(la, s), "logical score"); }
  } else {
    TargetArgs ta{};
    ta.U = (const double*)U_target; ta.n_targets = n_targets; ta.d = c->d;
    ta.st64 = (double*)at(L.st64);
    ta.st32 = c->prec == 32 ? (float*)at(L.st) : nullptr;
    HIPCHK(launch_targets(ta, s), "targets");
    if (c->real) HIPCHK(launch_tile_to_real(ta.st64, n_targets, c->d, ta.st32, s), "targets (real)");
  }
  const void* st_tiles = c->prec == 32 ? at(L.st) : at(L.st64);
  EnvArgs ev{};
  ev.prec = c->prec; ev.items = items; ev.n_items = (int)p.items.size();
  ev.chunk_item = (const int32_t*)at(L.chunk_item); ev.n_chunks_total = p.total_chunks;
  ev.pre = pre_cur; ev.suf = suf_cur; ev.st = st_tiles; ev.st64 = (const double*)at(L.st64);
  ev.env = grad ? at(L.env) : nullptr; ev.F = c->score_kind ? nullptr : F_items; ev.Fim = nullptr;
  ev.d = c->d; ev.f_by_src = grouped ? 0 : 1; ev.seed_by_item = c->score_kind ? 1 : 0;
  if (grad || !c->score_kind) { StageTimer t(c, 4, s); HIPCHK(launch_env(ev, s), "env"); }

  if (grad) {
    HIPCHK(launch_fill_int((int*)at(L.counters) + 16, 0, 16, s), "fill");
    sa.counter = (int*)at(L.counters) + 16;
    { StageTimer t(c, 5, s); HIPCHK(launch_slice_backward(c->prec, sa, grid, s), "backward"); }
    { StageTimer t(c, 6, s); HIPCHK(launch_traces(c->prec, sa, p.total_slices, s), "traces"); }
  }
  if (grad || grouped) {
    GradArgs ga{};
    ga.prec = c->prec; ga.gtrace = grad ? (const double*)at(L.gtrace) : nullptr;
    ga.amps = b->amps; ga.item_amp_offset = (const int64_t*)at(L.amp_off); ga.items = items;
    ga.n_items = (int)p.items.size(); ga.static_coef = b->static_coef; ga.ctrl_scale = b->ctrl_scale;
    ga.n_ctrl = c->nc; ga.n_static = c->ns; ga.order = c->order; ga.hold_foh = c->hold == LMAG_FOH;
    ga.nb = c->nb; ga.dt = b->dt;
    ga.inv_d2 = c->score_kind ? 1.0 : 1.0 / ((double)c->d * c->d);   // the seed carries its scale
    ga.grad = grad ? grad_out : nullptr;
    ga.group_first_item = grouped ? (const int32_t*)at(L.group_first) : nullptr;
    ga.group_items = grouped ? (const int32_t*)at(L.group_items) : nullptr;
    ga.n_groups = p.n_groups; ga.F_items = F_items; ga.F_out = grouped ? F_out : nullptr;
    ga.group_global = grouped ? (const int32_t*)at(L.group_global) : nullptr;
    if (!grad) {
      // group means of F only: reuse the grad kernel with a null gradient
      ga.gtrace = nullptr;
    }
    { StageTimer t(c, 7, s); HIPCHK(launch_grad(ga, grad ? p.max_slices : 1, s), "grad"); }
  }
  return LMAG_OK;
}

// Workspace of lmag_fidelity_and_grad_noalloc: a file-scope device array. Each
// GPU the library runs on holds its own copy, at its own address, until the
// process ends. Host code never passes the array's name to a kernel or copy (in
// host code it is a host-side stand-in); it uses the address that
// hipGetSymbolAddress returns with the device current, taken once per device.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 256;
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
char* g_scratch_addr[kMaxDevices] = {};

// Device address of this context's copy of `scratch` (the context's device must
// be current). Returns nullptr and leaves a message if the lookup fails.
char* scratch_address(lmag_ctx* c) {
  if (c->device < 0 || c->device >= kMaxDevices) {
    c->err = "device index beyond the scratch table";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[c->device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      c->err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_addr[c->device] = (char*)ptr;
  }
  return g_scratch_addr[c->device];
}

size_t device_budget(lmag_ctx* c) {
  if (c->ws_max) return c->ws_max;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) { (void)hipGetLastError(); return (size_t)64 << 30; }
  return (size_t)((double)(fr + c->ws_size) * 0.85);
}

// ---------------------------------------------------------------------------
// Block-tiled path (n = 64 T > 64): every per-slice stage is one batched launch
// over all slices (or over the active chunks of an ordered product step).
struct BigPlan {
  std::vector<int32_t> chain_slice, chain_chunk, chain_off;      // forward step k: [off[k], off[k+1])
  std::vector<int32_t> chain_zsrc, chain_zdst;                   // backward ping-pong indices (see run_big)
  std::vector<int32_t> odd_chunks, odd_off;                      // chunks of odd length, per window
  std::vector<int32_t> pl_cont_slice, pl_cont_next, pl_cont_off;  // forward step k, P_loc kept per
  std::vector<int32_t> pl_end_slice, pl_end_chunk, pl_end_off;    // slice (see run_big)
  std::vector<int32_t> scan_a, scan_b, scan_c, scan_off;         // per level, prefix then suffix
  std::vector<int32_t> copy_c, copy_off;                         // inactive entries per level
  std::vector<int32_t> env_suf_c, env_suf_next, env_nosuf_c;     // S_T^dag Suf_excl / S_T^dag
  std::vector<int32_t> env_suf_t, env_nosuf_t;                   // their targets
  std::vector<int32_t> env_pre_c, env_pre_prev, env_nopre_c;     // Pre_excl X / X
  std::vector<int32_t> item_last_chunk, item_target, item_src;
  std::vector<int32_t> ident;                                    // 0, 1, 2, ...
  int C = 0, levels = 0;
};

// Sparse tables of the 64 x 64 basis (host copy of the FP64 tiles): the union
// of the supports, numbered column by column (ascending rows), each position
// with its entries by ascending j; and the entries of each B_j with their
// position. Returns false (dense kernels) if a column has more than SP_COLCAP
// support rows.
bool build_sparse(lmag_ctx* c, const std::vector<double>& hb, int nb, int prec) {
  auto at = [&](int j, int x, int part) { return hb[((size_t)j * TILE + x) * 2 + part]; };
  auto nz = [&](int j, int x) { return at(j, x, 0) != 0.0 || at(j, x, 1) != 0.0; };
  std::vector<int16_t> cslot(TILE, -1);
  std::vector<int32_t> col_ptr(65, 0), sup_eptr(1, 0), ptr_j(nb + 1, 0);
  std::vector<uint8_t> sup_row, pe_j;
  std::vector<double> pe_v;
  int n_sup = 0;
  for (int col = 0; col < 64; ++col) {
    for (int row = 0; row < 64; ++row) {
      const int x = row * 64 + col;
      bool any = false;
      for (int j = 0; j < nb; ++j)
        if (nz(j, x)) {
          any = true;
          pe_j.push_back((uint8_t)j);
          pe_v.push_back(at(j, x, 0));
          pe_v.push_back(at(j, x, 1));
        }
      if (!any) continue;
      cslot[x] = (int16_t)n_sup++;
      sup_row.push_back((uint8_t)row);
      sup_eptr.push_back((int32_t)pe_j.size());
    }
    col_ptr[col + 1] = n_sup;
    if (col_ptr[col + 1] - col_ptr[col] > SP_COLCAP) return false;
  }
  const int nnz = (int)pe_j.size();
  if (nnz == 0) return false;
  // compact slots in register-tile order: thread t = 64 w + 16 g + cc holds
  // column 16 w + cc and rows 16 q + sub(g, r) in register 4 q + r
  std::vector<uint32_t> kpack(256);
  std::vector<int32_t> slot_of(TILE, -1);
  int next = 0;
  for (int t = 0; t < 256; ++t) {
    const int w = t >> 6, g = (t & 63) >> 4, cc = t & 15;
    uint32_t mask = 0;
    const int first = next;
    for (int q = 0; q < 4; ++q)
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * q + (prec == 32 ? 4 * g + r : g + 4 * r), col = 16 * w + cc;
        const int x = row * 64 + col;
        if (cslot[x] < 0) continue;
        mask |= 1u << (4 * q + r);
        slot_of[x] = next++;
      }
    kpack[t] = ((uint32_t)first << 16) | mask;
  }
  std::vector<uint16_t> ent_slot;
  std::vector<double> ent_v;
  for (int j = 0; j < nb; ++j) {
    for (int col = 0; col < 64; ++col)
      for (int row = 0; row < 64; ++row) {
        const int x = row * 64 + col;
        if (!nz(j, x)) continue;
        ent_slot.push_back((uint16_t)slot_of[x]);
        ent_v.push_back(at(j, x, 0));
        ent_v.push_back(at(j, x, 1));
      }
    ptr_j[j + 1] = (int32_t)ent_slot.size();
  }
  std::vector<char> blob;
  auto add = [&](const void* src, size_t bytes) {
    const size_t off = (blob.size() + 255) / 256 * 256;
    blob.resize(off + bytes);
    if (bytes) std::memcpy(blob.data() + off, src, bytes);
    return off;
  };
  auto addv = [&](const std::vector<double>& v) {
    if (prec == 64) return add(v.data(), v.size() * 8);
    std::vector<float> f(v.begin(), v.end());
    return add(f.data(), f.size() * 4);
  };
  const size_t o_cp = add(col_ptr.data(), col_ptr.size() * 4), o_sr = add(sup_row.data(), sup_row.size()),
               o_se = add(sup_eptr.data(), sup_eptr.size() * 4), o_pj = add(pe_j.data(), pe_j.size()),
               o_pv = addv(pe_v), o_ptr = add(ptr_j.data(), ptr_j.size() * 4),
               o_es = add(ent_slot.data(), ent_slot.size() * 2), o_ev = addv(ent_v),
               o_kp = add(kpack.data(), kpack.size() * 4);
  void* dev = nullptr;
  if (hipMalloc(&dev, blob.size()) != hipSuccess) { (void)hipGetLastError(); return false; }
  if (hipMemcpy(dev, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(dev);
    return false;
  }
  char* d = (char*)dev;
  c->sp_dev = dev;
  c->sp.n_sup = n_sup;
  c->sp.nnz = nnz;
  c->sp.col_ptr = (const int32_t*)(d + o_cp);
  c->sp.sup_row = (const uint8_t*)(d + o_sr);
  c->sp.sup_eptr = (const int32_t*)(d + o_se);
  c->sp.pe_j = (const uint8_t*)(d + o_pj);
  c->sp.pe_val = d + o_pv;
  c->sp.ptr_j = (const int32_t*)(d + o_ptr);
  c->sp.ent_slot = (const uint16_t*)(d + o_es);
  c->sp.ent_val = d + o_ev;
  c->sp.kpack = (const uint32_t*)(d + o_kp);
  return true;
}

// Chunk length of the block-tiled path: enough independent chunks (about 2048
// output tiles per chain step) to fill the device.
int big_auto_chunk(const lmag_ctx* c, long long total) {
  const long long Tn = c->n / 64;
  const long long want_chunks = std::max<long long>(1, 2048 / (Tn * Tn));
  return (int)std::max<long long>(1, (total + want_chunks - 1) / want_chunks);
}

// Layout of a block-tiled call: metadata and index lists, per-slice scalars,
// then the matrices. `window` is the number of slices whose per-slice matrices
// are held at once (all of them when the adjoint stores them).
struct BigLayout {
  size_t meta_end = 0, alpha = 0, gtrace = 0, ms = 0, nlev = 0, F_items = 0, part = 0, st64 = 0,
         st = 0, sq = 0, mlist = 0, mats = 0, cmats = 0, total = 0;
};

BigLayout big_layout(const lmag_ctx* c, size_t meta_bytes, int Ns, int Lc, int n_items, int window,
                     int n_targets, bool grad) {
  const int n = c->n, Tn = n / 64;
  const size_t mb = (size_t)n * n * (c->real ? 4 : 8);   // bytes per FP32 matrix
  BigLayout L;
  size_t o = align_up(meta_bytes);
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
  L.meta_end = o;
  const size_t planes = c->order == 6 ? 3 : 1;   // sixth order: a1, a2, a3 coefficients and traces
  L.alpha = take(planes * Ns * c->nb * 8);
  L.gtrace = take(planes * Ns * c->nb * 8);
  L.ms = take((size_t)Ns * 2);
  L.nlev = take((size_t)Ns);
  L.F_items = take((size_t)n_items * 8);
  L.part = take(std::max((size_t)window * Tn * n * 8, (size_t)window * Tn * Tn * c->nb * 8));
  // FP64 targets S_T^dag (complex; in the real basis followed by their real form)
  L.st64 = take((size_t)std::max(1, n_targets) * n * n * (c->real ? 24 : 16));
  L.st = take((size_t)std::max(1, n_targets) * mb);
  L.sq = take((size_t)Ns * kBigMaxSquarings * 4 + 4);   // squaring lists of every window
  L.mlist = take((size_t)Ns * 4 + 4);                    // slices by Pade degree, per window
  L.mats = take((size_t)(grad ? 11 : 7) * window * mb);
  L.cmats = take((size_t)8 * Lc * mb);
  L.total = o;
  return L;
}

// One slice window of a block-tiled call: whole chunks [c0, c1), slices
// [s0, s0 + ns), its chain steps, and the squaring lists read back after its
// slice exponents.
struct BigWindow {
  int c0 = 0, c1 = 0, s0 = 0, ns = 0;
  size_t koff = 0;                      // first entry of its chain-step offsets
  int smax = 0;
  size_t sq_base = 0;                   // first entry of its squaring lists
  std::vector<int32_t> sq_list, sq_off;
  int n2 = 0, n3 = 0;                   // slices at Pade degree 2 and 3 (lists at s0 of mlist)
  std::vector<int32_t> mlist_host;
};

lmag_status run_big(lmag_ctx* c, const lmag_batch* b, const int32_t* target_of_item,
                    int n_targets, bool grad, bool fidelity, const void* U_target, double* F_out,
                    void* grad_out, void* S_out, hipStream_t s) {
  const int n = c->n, Tn = n / 64;
  const size_t nn = (size_t)n * n, mb = nn * (c->real ? 4 : 8);   // FP32 matrices (real or complex)
  std::vector<int> all(b->n_items);
  for (int i = 0; i < b->n_items; ++i) all[i] = i;
  long long total = 0;
  for (int i = 0; i < b->n_items; ++i) total += b->n_slices[i];
  const int nt = fidelity ? n_targets : 0;
  const size_t budget = device_budget(c);
  // chunk length: enough independent chunks to fill the device in the chains;
  // product kernel: forced, else autotuned for this size, else the default
  int C_auto = c->chunk;
  int variant = c->big_variant >= 0 ? c->big_variant : kBigGemmDefault;
  const std::pair<int, int>* tuned = c->chunk <= 0 && c->big_variant < 0 ? tuned_for(c, total) : nullptr;
  if (tuned) { C_auto = tuned->first; variant = tuned->second; }
  if (C_auto <= 0) C_auto = big_auto_chunk(c, total);
  // metadata estimate (items, chunks, per-slice maps, index lists): bounded by
  // a few words per slice and chunk; the exact size is taken after planning
  auto plan_for = [&](int C, Plan& p) {
    p = Plan();
    const int saved = c->chunk;
    c->chunk = C;
    plan_wave(c, b, target_of_item, all, p, false);
    c->chunk = saved;
  };
  auto meta_estimate = [&](const Plan& p, int C) {
    return (size_t)p.items.size() * (sizeof(Item) + 64) + (size_t)p.chunks.size() * (sizeof(Chunk) + 64) +
           (size_t)p.total_slices * 16 + (size_t)std::max(1, (int)std::ceil(std::log2(std::max(2, p.max_chunks)))) *
           p.total_chunks * 32 + (size_t)(C + 2) * 64 + (1 << 16);
  };
  // stored: every slice's matrices at once; otherwise the largest window that
  // fits, with chunks no longer than the window
  Plan p;
  plan_for(C_auto, p);
  int W = p.total_slices;
  BigLayout BL = big_layout(c, meta_estimate(p, C_auto), p.total_slices, p.total_chunks,
                            (int)p.items.size(), W, nt, grad);
  if (BL.total > budget) {
    int lo = 0, hi = W;   // largest fitting window in (lo, hi]
    while (hi - lo > 1) {
      const int mid = lo + (hi - lo) / 2;
      Plan pm;
      const int Cm = std::min(C_auto, mid);
      plan_for(Cm, pm);
      const BigLayout Lm = big_layout(c, meta_estimate(pm, Cm), pm.total_slices, pm.total_chunks,
                                      (int)pm.items.size(), mid, nt, grad);
      if (Lm.total + ((size_t)1 << 20) <= budget) lo = mid; else hi = mid;
    }
    if (lo == 0)
      return c->fail(LMAG_E_NOMEM, "block-tiled call does not fit the workspace budget of " +
                                       std::to_string(budget) + " bytes even one slice at a time");
    W = lo;
    plan_for(std::min(C_auto, W), p);
  }
  const int Ns = p.total_slices, Lc = p.total_chunks, C = p.chunk_size;
  const bool windowed = W < Ns;
  // chunks in chain order, grouped into windows of whole chunks of at most W slices
  std::vector<Chunk> chs(Lc);
  for (const Chunk& ch : p.chunks) chs[ch.chunk] = ch;
  std::vector<BigWindow> win;
  for (int ci = 0; ci < Lc;) {
    BigWindow w;
    w.c0 = ci; w.s0 = chs[ci].first;
    int cnt = 0;
    while (ci < Lc && cnt + chs[ci].count <= W) cnt += chs[ci++].count;
    w.c1 = ci; w.ns = cnt;
    win.push_back(std::move(w));
  }
  BigPlan q;
  q.C = C;
  // chain steps per window: step k advances the window's chunks longer than k
  // (window-local slice index, global chunk index)
  // The chain products ping-pong between two per-chunk buffers instead of
  // copying back after every step. Forward: step k reads buffer k & 1 and
  // writes the other, so a chunk of length L ends in buffer L & 1 (chunks of
  // odd length are copied to buffer 0 once, at the end). Backward: the chunk's
  // suffix state starts in the environment array at its own last step; its
  // buffer at step k alternates with the steps it has taken, (L - 1 - k) & 1,
  // addressed through index lists into the adjacent environment (Lc + c) and
  // spare (c) arrays.
  // Where every slice's P_loc is kept (the adjoint's forward), step k instead
  // reads the P_loc - I of each chunk's k-th slice and writes that of its next
  // slice in place, or the chunk total at the chunk's last slice: no buffers
  // and no copies. pl_* hold those two lists per step (offsets parallel to
  // chain_off).
  q.odd_off.push_back(0);
  for (BigWindow& w : win) {
    w.koff = q.chain_off.size();
    q.chain_off.push_back((int32_t)q.chain_slice.size());
    q.pl_cont_off.push_back((int32_t)q.pl_cont_slice.size());
    q.pl_end_off.push_back((int32_t)q.pl_end_slice.size());
    for (int k = 0; k < C; ++k) {
      for (int ci = w.c0; ci < w.c1; ++ci)
        if (chs[ci].count > k) {
          const int sl = chs[ci].first + k - w.s0;
          q.chain_slice.push_back(sl);
          q.chain_chunk.push_back(ci);
          const bool in_env = ((chs[ci].count - 1 - k) & 1) == 0;
          q.chain_zsrc.push_back(in_env ? Lc + ci : ci);
          q.chain_zdst.push_back(in_env ? ci : Lc + ci);
          if (chs[ci].count > k + 1) {
            q.pl_cont_slice.push_back(sl);
            q.pl_cont_next.push_back(sl + 1);
          } else {
            q.pl_end_slice.push_back(sl);
            q.pl_end_chunk.push_back(ci);
          }
        }
      q.chain_off.push_back((int32_t)q.chain_slice.size());
      q.pl_cont_off.push_back((int32_t)q.pl_cont_slice.size());
      q.pl_end_off.push_back((int32_t)q.pl_end_slice.size());
    }
    for (int ci = w.c0; ci < w.c1; ++ci)
      if (chs[ci].count & 1) q.odd_chunks.push_back(ci);
    q.odd_off.push_back((int32_t)q.odd_chunks.size());
  }
  // scan levels: inclusive prefix P[c] = P[c] P[c - st]; suffix S[c] = S[c + st] S[c]
  q.scan_off.push_back(0);
  q.copy_off.push_back(0);
  for (int st = 1; st < p.max_chunks; st <<= 1, ++q.levels) {
    for (int dir = 0; dir < 2; ++dir) {
      for (int cidx = 0; cidx < Lc; ++cidx) {
        const Item& it = p.items[p.chunk_item[cidx]];
        const int lc = cidx - it.first_chunk;
        if (dir == 0 && lc >= st) { q.scan_a.push_back(cidx); q.scan_b.push_back(cidx - st); q.scan_c.push_back(cidx); }
        else if (dir == 1 && lc + st < it.n_chunks) { q.scan_a.push_back(cidx + st); q.scan_b.push_back(cidx); q.scan_c.push_back(cidx); }
        else q.copy_c.push_back(cidx);
      }
      q.scan_off.push_back((int32_t)q.scan_a.size());
      q.copy_off.push_back((int32_t)q.copy_c.size());
    }
  }
  for (int cidx = 0; cidx < Lc; ++cidx) {
    const Item& it = p.items[p.chunk_item[cidx]];
    const int lc = cidx - it.first_chunk;
    if (lc + 1 < it.n_chunks) {
      q.env_suf_c.push_back(cidx); q.env_suf_next.push_back(cidx + 1); q.env_suf_t.push_back(it.target);
    } else {
      q.env_nosuf_c.push_back(cidx); q.env_nosuf_t.push_back(it.target);
    }
    if (lc > 0) { q.env_pre_c.push_back(cidx); q.env_pre_prev.push_back(cidx - 1); }
    else q.env_nopre_c.push_back(cidx);
  }
  for (const Item& it : p.items) {
    q.item_last_chunk.push_back(it.first_chunk + it.n_chunks - 1);
    q.item_target.push_back(it.target);
    q.item_src.push_back(it.src);
  }
  for (int i = 0; i < std::max(Ns, Lc); ++i) q.ident.push_back(i);

  // ---- workspace: metadata, int lists, then scalars and matrices
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
  Layout L{};
  L.items = take(p.items.size() * sizeof(Item));
  L.chunks = take(p.chunks.size() * sizeof(Chunk));
  L.chunk_item = take(p.chunk_item.size() * 4);
  L.slice_item = take(p.slice_item.size() * 4);
  L.amp_off = take(p.amp_off.size() * 8);
  L.group_first = take(p.group_first.size() * 4);
  L.group_items = take(p.group_items.size() * 4);
  L.group_global = take(p.group_global.size() * 4);
  std::vector<std::pair<size_t, const std::vector<int32_t>*>> lists;
  auto list = [&](const std::vector<int32_t>& v) { size_t r = take(v.size() * 4 + 4); lists.push_back({r, &v}); return r; };
  const size_t o_cs = list(q.chain_slice), o_cc = list(q.chain_chunk), o_sa = list(q.scan_a),
               o_sb = list(q.scan_b), o_sc = list(q.scan_c), o_cp = list(q.copy_c),
               o_es = list(q.env_suf_c), o_en = list(q.env_suf_next), o_ens = list(q.env_nosuf_c),
               o_ep = list(q.env_pre_c), o_epp = list(q.env_pre_prev), o_enp = list(q.env_nopre_c),
               o_est = list(q.env_suf_t), o_ent = list(q.env_nosuf_t),
               o_il = list(q.item_last_chunk), o_it = list(q.item_target),
               o_is = list(q.item_src), o_id = list(q.ident), o_zs = list(q.chain_zsrc),
               o_zd = list(q.chain_zdst), o_od = list(q.odd_chunks),
               o_pcs = list(q.pl_cont_slice), o_pcn = list(q.pl_cont_next),
               o_pes = list(q.pl_end_slice), o_pec = list(q.pl_end_chunk);
  BL = big_layout(c, o, Ns, Lc, (int)p.items.size(), W, nt, grad);
  L.meta_end = BL.meta_end;
  if (BL.total > budget)
    return c->fail(LMAG_E_NOMEM, "block-tiled call needs " + std::to_string(BL.total) +
                                     " bytes of workspace, over the budget of " + std::to_string(budget));
  lmag_status st = ensure_ws(c, BL.total);
  if (st != LMAG_OK) return st;
  // upload metadata + lists in one copy
  st = ensure_pinned(c, L.meta_end);
  if (st != LMAG_OK) return st;
  std::memset(c->pinned, 0, L.meta_end);
  auto put = [&](size_t off, const void* src, size_t bytes) { if (bytes) std::memcpy(c->pinned + off, src, bytes); };
  put(L.items, p.items.data(), p.items.size() * sizeof(Item));
  put(L.chunks, p.chunks.data(), p.chunks.size() * sizeof(Chunk));
  put(L.chunk_item, p.chunk_item.data(), p.chunk_item.size() * 4);
  put(L.slice_item, p.slice_item.data(), p.slice_item.size() * 4);
  put(L.amp_off, p.amp_off.data(), p.amp_off.size() * 8);
  put(L.group_first, p.group_first.data(), p.group_first.size() * 4);
  put(L.group_items, p.group_items.data(), p.group_items.size() * 4);
  put(L.group_global, p.group_global.data(), p.group_global.size() * 4);
  for (auto& l : lists) put(l.first, l.second->data(), l.second->size() * 4);
  HIPCHK(hipMemcpyAsync(c->ws, c->pinned, L.meta_end, hipMemcpyHostToDevice, s), "plan upload");
  HIPCHK(hipEventRecord(c->upload_done, s), "event");
  c->upload_pending = true;

  char* w_ = c->ws;
  auto at = [&](size_t off) { return (void*)(w_ + off); };
  auto ip = [&](size_t off) { return (const int32_t*)(w_ + off); };
  auto M = [&](int k) { return at(BL.mats + (size_t)k * W * mb); };     // per-slice matrix array k (window)
  auto CM = [&](int k) { return at(BL.cmats + (size_t)k * Lc * mb); };  // per-chunk matrix array k
  void *A = M(0), *A2 = M(1), *R0 = M(2), *S = M(3), *Qi = M(4), *T1 = M(5), *T2 = M(6);
  void *Pl = grad ? M(7) : nullptr, *Em = grad ? M(8) : nullptr, *T3 = grad ? M(9) : nullptr,
       *T4 = grad ? M(10) : nullptr;
  const Item* items = (const Item*)at(L.items);
  int8_t* ms_all = (int8_t*)at(BL.ms);
  int8_t* nlev_all = (int8_t*)at(BL.nlev);

  auto gemm = [&](int batch, const void* Ap, const int32_t* Ai, const void* Bp, const int32_t* Bi,
                  const void* Cp, const int32_t* Ci, double alpha, const void* Dp = nullptr,
                  const int32_t* Di = nullptr, double beta = 0.0, double gamma = 0.0, int tA = 0,
                  int tB = 0, const int8_t* pred = nullptr, int thresh = 0) {
    BigGemmArgs g{};
    g.n = n; g.batch = batch; g.A = Ap; g.Ai = Ai; g.B = Bp; g.Bi = Bi; g.C = Cp; g.Ci = Ci;
    g.D = Dp; g.Di = Di; g.alpha = alpha; g.beta = beta; g.gamma = gamma; g.transA = tA; g.transB = tB;
    g.pred = pred; g.pred_stride = 1; g.pred_thresh = thresh; g.variant = variant;
    return c->real ? launch_rgemm(g, s) : launch_bgemm(32, g, s);
  };
  // C = alpha A B + beta D + beta2 D2 with index maps (null: the batch index)
  auto gemmx = [&](int batch, const void* Ap, const int32_t* Ai, const void* Bp, const int32_t* Bi,
                   const void* Cp, const int32_t* Ci, double alpha, const void* Dp, const int32_t* Di,
                   double beta, const void* D2p, const int32_t* D2i, double beta2,
                   const int8_t* pred = nullptr, int thresh = 0) {
    BigGemmArgs g{};
    g.n = n; g.batch = batch; g.A = Ap; g.Ai = Ai; g.B = Bp; g.Bi = Bi; g.C = Cp; g.Ci = Ci;
    g.D = Dp; g.Di = Di; g.D2 = D2p; g.D2i = D2i;
    g.alpha = alpha; g.beta = beta; g.beta2 = beta2;
    g.pred = pred; g.pred_stride = 1; g.pred_thresh = thresh; g.variant = variant;
    return c->real ? launch_rgemm(g, s) : launch_bgemm(32, g, s);
  };
  auto gemm2 = [&](int batch, const void* Ap, const void* Bp, const void* Cp, double alpha,
                   const void* Dp, double beta, const void* D2p, double beta2,
                   const int8_t* pred = nullptr, int thresh = 0) {
    return gemmx(batch, Ap, nullptr, Bp, nullptr, Cp, nullptr, alpha, Dp, nullptr, beta, D2p, nullptr,
                 beta2, pred, thresh);
  };
  // C = alpha A B + beta D and, from the same tiles, C2 = c2c C + c2e E2 + c2g I
  auto gemm_dual = [&](int batch, const void* Ap, const int32_t* Ai, const void* Bp, const int32_t* Bi,
                       const void* Cp, const int32_t* Ci, double alpha, const void* Dp, const int32_t* Di,
                       double beta, const void* C2p, const int32_t* C2i, double c2c, const void* E2p,
                       const int32_t* E2i, double c2e, double c2g) {
    BigGemmArgs g{};
    g.n = n; g.batch = batch; g.A = Ap; g.Ai = Ai; g.B = Bp; g.Bi = Bi; g.C = Cp; g.Ci = Ci;
    g.D = Dp; g.Di = Di; g.alpha = alpha; g.beta = beta; g.variant = variant;
    g.C2 = C2p; g.C2i = C2i; g.E2 = E2p; g.E2i = E2i; g.c2_c = c2c; g.c2_e = c2e; g.c2_gamma = c2g;
    return c->real ? launch_rgemm(g, s) : launch_bgemm(32, g, s);
  };
  auto axpby = [&](int batch, const void* X, const int32_t* Xi, void* Y, const int32_t* Yi, double a,
                   const void* Z = nullptr, const int32_t* Zi = nullptr, double cc = 0.0, double d = 0.0,
                   const int8_t* ms = nullptr) {
    BigAxpbyArgs g{};
    g.n = n; g.batch = batch; g.X = X; g.Xi = Xi; g.Z = Z; g.Zi = Zi; g.Y = Y; g.Yi = Yi;
    g.a = a; g.c = cc; g.d = d; g.ms = ms;
    return c->real ? launch_raxpby(g, s) : launch_baxpby(32, g, s);
  };
  const double* b3 = c->pade.b3;

  // ---- coefficients of every slice
  AlphaArgs aa{};
  aa.prec = 32; aa.amps = b->amps; aa.item_amp_offset = (const int64_t*)at(L.amp_off);
  aa.items = items; aa.n_items = (int)p.items.size(); aa.static_coef = b->static_coef;
  aa.ctrl_scale = b->ctrl_scale; aa.n_ctrl = c->nc; aa.n_static = c->ns; aa.order = c->order;
  aa.hold_foh = c->hold == LMAG_FOH; aa.nb = c->nb; aa.dt = b->dt;
  aa.slice_item = (const int32_t*)at(L.slice_item); aa.alpha = (double*)at(BL.alpha);
  aa.n_slices_total = Ns;
  { StageTimer t(c, 0, s); HIPCHK(c->order == 6 ? launch_alpha6(aa, s) : launch_alpha(aa, s), "alpha"); }
  const size_t coef_plane = (size_t)Ns * c->nb;
  // sixth order: a1, a2, a3 of the window's slices on the order-1 basis (in
  // A2, R0, S), then C1 = [a1, a2] (in Qi), W = 2 a3 + C1 (in T2),
  // C2 = -(1/60) [a1, W] and Y = a2 + C2 (in T1), X = C1 - 20 a1 - a3 (in Qi);
  // `tmp` is a free array
  auto order6_levels = [&](const BigWindow& w, void* tmp) -> lmag_status {
    const int Wn = w.ns;
    const double* coef = (const double*)at(BL.alpha) + (size_t)w.s0 * c->nb;
    void* al[3] = {A2, R0, S};
    for (int pl = 0; pl < 3; ++pl) {
      BigOmegaArgs oa{};
      oa.n = n; oa.n_slices = Wn; oa.nb = c->nb; oa.basis = c->basis32;
      oa.tile_ptr = c->tile_ptr; oa.tile_j = c->tile_j;
      oa.alpha = coef + pl * coef_plane; oa.omega = al[pl]; oa.part = (double*)at(BL.part);
      HIPCHK(c->real ? launch_romega(oa, s) : launch_bomega(32, oa, s), "a_p");
    }
    HIPCHK(gemm(Wn, A2, nullptr, R0, nullptr, T1, nullptr, 1.0), "a1 a2");
    HIPCHK(gemm(Wn, R0, nullptr, A2, nullptr, Qi, nullptr, -1.0, T1, nullptr, 1.0), "C1");
    HIPCHK(axpby(Wn, S, nullptr, T2, nullptr, 2.0, Qi, nullptr, 1.0), "W");
    HIPCHK(gemm(Wn, A2, nullptr, T2, nullptr, tmp, nullptr, 1.0), "a1 W");
    HIPCHK(gemm(Wn, T2, nullptr, A2, nullptr, T1, nullptr, 1.0 / 60.0, tmp, nullptr, -1.0 / 60.0), "C2");
    HIPCHK(axpby(Wn, A2, nullptr, Qi, nullptr, -20.0, Qi, nullptr, 1.0), "X");
    HIPCHK(axpby(Wn, S, nullptr, Qi, nullptr, -1.0, Qi, nullptr, 1.0), "X");
    HIPCHK(axpby(Wn, R0, nullptr, T1, nullptr, 1.0, T1, nullptr, 1.0), "Y");
    return LMAG_OK;
  };
  c->last_ms = ms_all;
  c->last_total_slices = Ns;

  // Forward of one window: exponents, Pade 3 with the Neumann inverse,
  // squarings, then the chain of its chunks (storing P_loc when asked).
  // Matrices near the identity are carried as I + X with only X inside the
  // products (see the 64 x 64 slice kernel): P = I + X_P, Q = I - E,
  // Q^{-1} = I + X_Q, r = I + D. The first pass over a window reads its
  // scaling exponents back to size the squaring loop (one host wait).
  void* Pc[2] = {CM(0), CM(1)};
  auto forward_window = [&](BigWindow& w, bool first_pass, bool store_ploc) -> lmag_status {
    const int Wn = w.ns;
    int8_t* ms_w = ms_all + 2 * (size_t)w.s0;
    int8_t* nlev_w = nlev_all + w.s0;
    BigOmegaArgs om{};
    om.n = n; om.n_slices = Wn; om.nb = c->nb; om.basis = c->basis32;
    om.tile_ptr = c->tile_ptr; om.tile_j = c->tile_j;
    om.alpha = (const double*)at(BL.alpha) + (size_t)w.s0 * c->nb;
    om.omega = A; om.part = (double*)at(BL.part); om.ms = ms_w; om.nlev = nlev_w;
    for (int i = 0; i < 4; ++i) om.b3[i] = b3[i];
    if (c->order == 6) {
      // Omega = a1 + a3 / 12 + (1/240) [X, Y]
      StageTimer t(c, 1, s);
      lmag_status st6 = order6_levels(w, A);
      if (st6 != LMAG_OK) return st6;
      HIPCHK(gemm(Wn, Qi, nullptr, T1, nullptr, T2, nullptr, 1.0), "X Y");
      HIPCHK(gemm(Wn, T1, nullptr, Qi, nullptr, A, nullptr, -1.0 / 240.0, T2, nullptr, 1.0 / 240.0), "[X, Y]");
      HIPCHK(axpby(Wn, A2, nullptr, A, nullptr, 1.0, A, nullptr, 1.0), "+ a1");
      HIPCHK(axpby(Wn, S, nullptr, A, nullptr, 1.0 / 12.0, A, nullptr, 1.0), "+ a3 / 12");
      HIPCHK(c->real ? launch_rnorm_dense(om, s) : launch_bnorm_dense(32, om, s), "omega norm");
    } else {
      StageTimer t(c, 1, s);
      HIPCHK(c->real ? launch_romega(om, s) : launch_bomega(32, om, s), "omega");
    }
    if (first_pass) {
      std::vector<int8_t> msh((size_t)Wn * 2);
      HIPCHK(hipMemcpyAsync(msh.data(), ms_w, msh.size(), hipMemcpyDeviceToHost, s), "ms");
      HIPCHK(hipStreamSynchronize(s), "sync");
      w.smax = 0;
      for (int i = 0; i < Wn; ++i) w.smax = std::max<int>(w.smax, msh[2 * i + 1]);
      if (w.smax > kBigMaxSquarings)
        return c->fail(LMAG_E_UNSUPPORTED, "a slice exponent needs more than " +
                                               std::to_string(kBigMaxSquarings) + " squarings");
      // per-k lists of the window's slices that take a k-th squaring
      w.sq_list.clear();
      w.sq_off.assign(1, 0);
      for (int k = 0; k < w.smax; ++k) {
        for (int i = 0; i < Wn; ++i)
          if (msh[2 * i + 1] > k) w.sq_list.push_back(i);
        w.sq_off.push_back((int32_t)w.sq_list.size());
      }
      w.sq_base = 0;
      for (const BigWindow& v : win) {
        if (&v == &w) break;
        w.sq_base += v.sq_list.size();
      }
      if (!w.sq_list.empty())
        HIPCHK(hipMemcpyAsync((int32_t*)at(BL.sq) + w.sq_base, w.sq_list.data(), w.sq_list.size() * 4,
                              hipMemcpyHostToDevice, s), "squaring lists");
      // the window's slices at Pade degree 2 (by the degree-4 series of r_2),
      // then those at degree 3
      std::vector<int32_t> ml;
      for (int i = 0; i < Wn; ++i)
        if (msh[2 * i] == 2) ml.push_back(i);
      w.n2 = (int)ml.size();
      for (int i = 0; i < Wn; ++i)
        if (msh[2 * i] != 2) ml.push_back(i);
      w.n3 = Wn - w.n2;
      w.mlist_host.swap(ml);
      HIPCHK(hipMemcpyAsync((int32_t*)at(BL.mlist) + w.s0, w.mlist_host.data(), (size_t)Wn * 4,
                            hipMemcpyHostToDevice, s), "degree lists");
    }
    const int32_t* sq = ip(BL.sq) + w.sq_base;
    const int32_t* L2 = ip(BL.mlist) + w.s0;     // degree-2 slices (window-local)
    const int32_t* L3 = L2 + w.n2;               // degree-3 slices
    {
      StageTimer t(c, 2, s);
      if (w.n3) {
        const int n3 = w.n3;
        HIPCHK(gemm(n3, A, L3, A, L3, A2, L3, 1.0), "A2");
        HIPCHK(axpby(n3, A2, L3, T1, L3, b3[3], nullptr, nullptr, 0.0, b3[1]), "W");
        HIPCHK(gemm(n3, A, L3, T1, L3, T2, L3, 1.0), "U");                                    // T2 = U
        HIPCHK(axpby(n3, A2, L3, T1, L3, b3[2], T2, L3, 1.0), "X_P");                         // T1 = b2 A2 + U
        HIPCHK(axpby(n3, A2, L3, S, L3, -b3[2], T2, L3, 1.0), "E");                          // S = E = U - b2 A2
        HIPCHK(axpby(n3, S, L3, T2, L3, 1.0), "X = E");                                       // T2 = X
        // (I + X)(I + F2) - I = X + F2 + F2 X; level k runs for the slices whose
        // Neumann level count exceeds k (the others copy F and X through)
        void *F = S, *X = T2, *F2 = R0, *Xn = Qi;
        for (int k = 1; k < kBigNeumannLevels; ++k) {
          HIPCHK(gemm(n3, F, L3, F, L3, F2, L3, 1.0, nullptr, nullptr, 0.0, 0.0, 0, 0, nlev_w, k), "F2");
          HIPCHK(gemmx(n3, F2, L3, X, L3, Xn, L3, 1.0, X, L3, 1.0, F2, L3, 1.0, nlev_w, k), "X + F2 + F2 X");
          std::swap(F, F2);
          std::swap(X, Xn);
        }
        if (X != Qi) HIPCHK(axpby(n3, X, L3, Qi, L3, 1.0), "X_Q");
        HIPCHK(gemmx(n3, Qi, L3, T1, L3, R0, L3, 1.0, Qi, L3, 1.0, T1, L3, 1.0), "D");   // R0 = X_Q + X_P + X_Q X_P
        HIPCHK(axpby(n3, R0, L3, S, L3, 1.0), "S");
      }
      if (w.n2) {
        // Pade 2 by its power series cut at degree 4 (the degree-4 Taylor
        // polynomial): D = A + A^2 (I/2 + A/6 + A^2/24); s = 0 at this degree
        const int n2 = w.n2;
        // (no squarings at this degree and the adjoint reads neither R0 nor a
        // second copy of D here: D goes straight to S; T1 = W stays for the
        // adjoint)
        HIPCHK(gemm_dual(n2, A, L2, A, L2, A2, L2, 1.0, nullptr, nullptr, 0.0, T1, L2, 1.0 / 24.0, A, L2,
                         1.0 / 6.0, 0.5), "A2, W = I/2 + A/6 + A2/24");
        HIPCHK(gemm(n2, A2, L2, T1, L2, S, L2, 1.0, A, L2, 1.0), "D");
      }
      // (I + D)^2 = I + 2 D + D^2
      for (int k = 0; k < w.smax; ++k) {
        const int cnt = w.sq_off[k + 1] - w.sq_off[k];
        const int32_t* li = sq + w.sq_off[k];
        if (!cnt) continue;
        HIPCHK(gemm(cnt, S, li, S, li, T1, li, 1.0, S, li, 2.0), "square");
        HIPCHK(axpby(cnt, T1, li, S, li, 1.0), "square copy");
      }
    }
    // ordered products inside the window's chunks, kept as M - I:
    // (I + D)(I + Q) - I = Q + D + D Q
    if (store_ploc) {
      // every slice's P_loc - I in place (Pl), the chunk totals into Pc[0]
      StageTimer t(c, 2, s);
      const int f0 = q.chain_off[w.koff], nf = q.chain_off[w.koff + 1] - f0;
      HIPCHK(axpby(nf, Pl, ip(o_cs) + f0, Pl, ip(o_cs) + f0, 0.0), "P_loc - I = 0");
      for (int k = 0; k < C; ++k) {
        const int a0 = q.pl_cont_off[w.koff + k], na = q.pl_cont_off[w.koff + k + 1] - a0;
        const int e0 = q.pl_end_off[w.koff + k], ne = q.pl_end_off[w.koff + k + 1] - e0;
        if (na) {
          const int32_t* sl = ip(o_pcs) + a0;
          HIPCHK(gemmx(na, S, sl, Pl, sl, Pl, ip(o_pcn) + a0, 1.0, Pl, sl, 1.0, S, sl, 1.0), "chain");
        }
        if (ne) {
          const int32_t* sl = ip(o_pes) + e0;
          HIPCHK(gemmx(ne, S, sl, Pl, sl, Pc[0], ip(o_pec) + e0, 1.0, Pl, sl, 1.0, S, sl, 1.0), "chain end");
        }
      }
      return LMAG_OK;
    }
    {
      StageTimer t(c, 2, s);
      HIPCHK(axpby(w.c1 - w.c0, Pc[0], ip(o_id) + w.c0, Pc[0], ip(o_id) + w.c0, 0.0), "P - I = 0");
      for (int k = 0; k < C; ++k) {
        const int a0 = q.chain_off[w.koff + k], cnt = q.chain_off[w.koff + k + 1] - a0;
        if (cnt == 0) continue;
        const int32_t* sl = ip(o_cs) + a0;
        const int32_t* chn = ip(o_cc) + a0;
        void* cur = Pc[k & 1];
        void* nxt = Pc[(k + 1) & 1];
        HIPCHK(gemmx(cnt, S, sl, cur, chn, nxt, chn, 1.0, cur, chn, 1.0, S, sl, 1.0), "chain");
      }
      const size_t wi = &w - win.data();
      const int od0 = q.odd_off[wi], nod = q.odd_off[wi + 1] - od0;
      if (nod) HIPCHK(axpby(nod, Pc[1], ip(o_od) + od0, Pc[0], ip(o_od) + od0, 1.0), "odd chunks");
    }
    return LMAG_OK;
  };
  const bool store_now = grad && !windowed;
  for (BigWindow& w : win) {
    st = forward_window(w, true, store_now);
    if (st != LMAG_OK) return st;
  }
  // ---- scan over chunk totals
  void* pre[2] = {CM(2), CM(3)};
  void* suf[2] = {CM(4), CM(5)};
  const void* pre_cur = Pc[0];
  const void* suf_cur = Pc[0];
  {
    StageTimer t(c, 3, s);
    int bsel = 0;
    for (int lv = 0; lv < q.levels; ++lv) {
      for (int dir = 0; dir < 2; ++dir) {
        if (dir == 1 && !grad) continue;
        const int li = 2 * lv + dir;
        const int a0 = q.scan_off[li], cnt = q.scan_off[li + 1] - a0;
        const int c0 = q.copy_off[li], ccnt = q.copy_off[li + 1] - c0;
        const void* in = dir == 0 ? pre_cur : suf_cur;
        void* out = dir == 0 ? pre[bsel] : suf[bsel];
        if (cnt)
          HIPCHK(gemmx(cnt, in, ip(o_sa) + a0, in, ip(o_sb) + a0, out, ip(o_sc) + a0, 1.0, in,
                       ip(o_sa) + a0, 1.0, in, ip(o_sb) + a0, 1.0), "scan");
        if (ccnt) HIPCHK(axpby(ccnt, in, ip(o_cp) + c0, out, ip(o_cp) + c0, 1.0), "scan copy");
      }
      pre_cur = pre[bsel];
      if (grad) suf_cur = suf[bsel];
      bsel ^= 1;
    }
  }
  auto finish_plan = [&]() {
    c->plan_info[0] = Ns; c->plan_info[1] = Lc; c->plan_info[2] = C; c->plan_info[3] = 0;
    c->plan_info[4] = (int64_t)BL.total;
    c->plan_recompute = grad && windowed;
    c->plan_waves = (int)win.size();
  };
  if (S_out) {   // U of every item = I + inclusive prefix at its last chunk
    if (c->real)   // back to column stacking: T^dag (I + R) T
      HIPCHK(launch_from_real((const float*)pre_cur, ip(o_il), c->d, (int)p.items.size(), S_out, ip(o_is), s),
             "extract");
    else
      HIPCHK(axpby((int)p.items.size(), pre_cur, ip(o_il), S_out, ip(o_is), 1.0, nullptr, nullptr, 0.0, 1.0),
             "extract");
  }
  if (!fidelity) { finish_plan(); return LMAG_OK; }
  // ---- targets, fidelity, environments
  // S_T^dag of every target (FP64 and FP32); in the real basis R_T^T = T S_T^dag T^dag
  double* st64 = (double*)at(BL.st64);
  if (c->real) {
    double* r64 = st64 + (size_t)std::max(1, n_targets) * nn * 2;
    HIPCHK(launch_btargets((const double*)U_target, n_targets, c->d, st64, nullptr, s), "targets");
    HIPCHK(launch_to_real(st64, c->d, n_targets, r64, s), "targets (real)");
    HIPCHK(launch_rcast(r64, (float*)at(BL.st), (size_t)n_targets * nn, s), "targets (FP32)");
    st64 = r64;
  } else {
    HIPCHK(launch_btargets((const double*)U_target, n_targets, c->d, st64, (float*)at(BL.st), s), "targets");
  }
  const bool grouped = p.n_groups > 0;
  double* F_items = grouped ? (double*)at(BL.F_items) : F_out;
  {
    StageTimer t(c, 4, s);
    BigFidArgs fa{};
    fa.n = n; fa.n_items = (int)p.items.size(); fa.d = c->d; fa.U = pre_cur; fa.U_index = ip(o_il);
    fa.st64 = st64; fa.target = ip(o_it); fa.F = F_items;
    fa.F_index = grouped ? nullptr : ip(o_is);
    HIPCHK(c->real ? launch_rfidelity(fa, s) : launch_bfidelity(32, fa, s), "fidelity");
  }
  if (grad) {
    void* X = CM(6);
    void* env = CM(7);
    {
      StageTimer t(c, 4, s);
      const void* stt = at(BL.st);
      if (!q.env_suf_c.empty())
        HIPCHK(gemm((int)q.env_suf_c.size(), stt, ip(o_est), suf_cur, ip(o_en), X, ip(o_es), 1.0, stt,
                    ip(o_est), 1.0), "env X");   // S_T^dag (I + Suf)
      if (!q.env_nosuf_c.empty())
        HIPCHK(axpby((int)q.env_nosuf_c.size(), stt, ip(o_ent), X, ip(o_ens), 1.0), "env X copy");
      if (!q.env_pre_c.empty())
        HIPCHK(gemm((int)q.env_pre_c.size(), pre_cur, ip(o_epp), X, ip(o_ep), env, ip(o_ep), 1.0, X,
                    ip(o_ep), 1.0), "env W");   // (I + Pre) X
      if (!q.env_nopre_c.empty())
        HIPCHK(axpby((int)q.env_nopre_c.size(), X, ip(o_enp), env, ip(o_enp), 1.0), "env W copy");
    }
    // ---- adjoint, window by window (last first). A windowed call re-runs the
    // window's forward first (recomputation instead of storage: the chunk
    // totals and environments are already known, only P_loc, D, Q^{-1}, A and
    // A^2 of its slices are rebuilt, bitwise as in the first pass).
    for (int wi = (int)win.size() - 1; wi >= 0; --wi) {
      BigWindow& w = win[wi];
      const int Wn = w.ns;
      if (windowed) {
        st = forward_window(w, false, true);
        if (st != LMAG_OK) return st;
      }
      const int32_t* sq = ip(BL.sq) + w.sq_base;
      {
        StageTimer t(c, 5, s);
        // backward chain: M_n = P_loc,n Z, Z <- Z S_n = Z + Z D_n (normal orientation)
        void* Zb = X;   // X (index c) and env (index Lc + c) are adjacent arrays
        for (int k = C - 1; k >= 0; --k) {
          const int a0 = q.chain_off[w.koff + k], cnt = q.chain_off[w.koff + k + 1] - a0;
          if (cnt == 0) continue;
          const int32_t* sl = ip(o_cs) + a0;
          const int32_t* zs = ip(o_zs) + a0;
          const int32_t* zd = ip(o_zd) + a0;
          HIPCHK(gemm(cnt, Pl, sl, Zb, zs, Em, sl, 1.0, Zb, zs, 1.0), "M");   // (I + Pl) Z
          if (k > 0) HIPCHK(gemm(cnt, Zb, zs, S, sl, Zb, zd, 1.0, Zb, zs, 1.0), "Z");
        }
        // Frechet derivative of the scaled Pade approximant at A in direction E = M / 2^s
        if (w.smax > 0) {   // E / 2^s on the slices with s > 0 (the first squaring list)
          const int32_t* l0 = ip(BL.sq) + w.sq_base;
          HIPCHK(axpby(w.sq_off[1], Em, l0, Em, l0, 1.0, nullptr, nullptr, 0.0, 0.0,
                       ms_all + 2 * (size_t)w.s0), "E scale");
        }
        const int32_t* L2 = ip(BL.mlist) + w.s0;
        const int32_t* L3 = L2 + w.n2;
        if (w.n3) {
          const int n3 = w.n3;
          HIPCHK(gemm(n3, A, L3, Em, L3, T1, L3, 1.0), "AE");
          HIPCHK(gemm(n3, Em, L3, A, L3, T1, L3, 1.0, T1, L3, 1.0), "L2");                    // T1 = L2
          HIPCHK(axpby(n3, A2, L3, T2, L3, b3[3], nullptr, nullptr, 0.0, b3[1]), "W");         // T2 = W
          HIPCHK(axpby(n3, T1, L3, T3, L3, b3[3]), "LW");                                       // T3 = L_W
          HIPCHK(gemm(n3, A, L3, T3, L3, T4, L3, 1.0), "A LW");
          HIPCHK(gemm(n3, Em, L3, T2, L3, T4, L3, 1.0, T4, L3, 1.0), "LU");                    // T4 = L_U
          HIPCHK(axpby(n3, T1, L3, T3, L3, b3[2], T4, L3, -1.0), "LQ");                        // T3 = L_Q
          HIPCHK(axpby(n3, T1, L3, T2, L3, b3[2], T4, L3, 1.0), "LP");                         // T2 = L_P
          // r = I + D (R0 = D), Q^{-1} = I + X_Q (Qi = X_Q)
          HIPCHK(gemmx(n3, T3, L3, R0, L3, T1, L3, -1.0, T2, L3, 1.0, T3, L3, -1.0), "X");   // T1 = L_P - L_Q - L_Q D
          HIPCHK(gemm(n3, Qi, L3, T1, L3, T3, L3, 1.0, T1, L3, 1.0), "K");                    // T3 = K
        }
        if (w.n2) {
          // derivative of the degree-4 polynomial A + A^2/2 + A^3/6 + A^4/24:
          // K = E + L2/2 + L2 (A/6 + A^2/24) + A^2 (E/6 + L2/24), L2 = A E + E A
          const int n2 = w.n2;
          // with W = I/2 + A/6 + A^2/24 (T1, kept from the forward):
          // K = E + L2 W + A^2 (E/6 + L2/24)
          HIPCHK(gemm(n2, A, L2, Em, L2, T3, L2, 1.0), "AE");
          HIPCHK(gemm_dual(n2, Em, L2, A, L2, T3, L2, 1.0, T3, L2, 1.0, T2, L2, 1.0 / 24.0, Em, L2, 1.0 / 6.0,
                           0.0), "L2, E/6 + L2/24");                                       // T3 = L2, T2
          HIPCHK(gemm(n2, T3, L2, T1, L2, T4, L2, 1.0, Em, L2, 1.0), "E + L2 W");
          HIPCHK(gemm(n2, A2, L2, T2, L2, T3, L2, 1.0, T4, L2, 1.0), "K");                    // T3 = K
        }
        // squaring recurrence K <- R K + K R = 2 K + D K + K D, D <- 2 D + D D for the
        // slices with s > k
        for (int k = 0; k < w.smax; ++k) {
          const int cnt = w.sq_off[k + 1] - w.sq_off[k];
          const int32_t* li = sq + w.sq_off[k];
          if (!cnt) continue;
          HIPCHK(gemm(cnt, R0, li, T3, li, T4, li, 1.0, T3, li, 2.0), "2K + DK");
          HIPCHK(gemm(cnt, T3, li, R0, li, T2, li, 1.0, T4, li, 1.0), "+ KD");
          HIPCHK(gemm(cnt, R0, li, R0, li, T1, li, 1.0, R0, li, 2.0), "2D + D^2");
          HIPCHK(axpby(cnt, T2, li, T3, li, 1.0), "K");
          HIPCHK(axpby(cnt, T1, li, R0, li, 1.0), "R");
        }
      }
      if (c->order == 6) {
        // cotangents of a1, a2, a3 from K = dF/dOmega through
        // Omega = a1 + a3/12 + [X, Y]/240, X = C1 - 20 a1 - a3, Y = a2 + C2,
        // C2 = -(1/60)[a1, W], W = 2 a3 + C1, C1 = [a1, a2]; for C = [P, Q]
        // with cotangent G the cotangents are [Q, G] for P and [G, P] for Q
        StageTimer t(c, 5, s);
        lmag_status st6 = order6_levels(w, A);
        if (st6 != LMAG_OK) return st6;
        // G_X = [Y, K] / 240 (S), G_Y = [K, X] / 240 (Pl)
        HIPCHK(gemm(Wn, T1, nullptr, T3, nullptr, Em, nullptr, 1.0), "Y K");
        HIPCHK(gemm(Wn, T3, nullptr, T1, nullptr, S, nullptr, -1.0 / 240.0, Em, nullptr, 1.0 / 240.0), "G_X");
        HIPCHK(gemm(Wn, T3, nullptr, Qi, nullptr, Em, nullptr, 1.0), "K X");
        HIPCHK(gemm(Wn, Qi, nullptr, T3, nullptr, Pl, nullptr, -1.0 / 240.0, Em, nullptr, 1.0 / 240.0), "G_Y");
        // G_a1 = K - 20 G_X (Qi), G_a3 = K / 12 - G_X (T1)
        HIPCHK(axpby(Wn, T3, nullptr, Qi, nullptr, 1.0, S, nullptr, -20.0), "G_a1");
        HIPCHK(axpby(Wn, T3, nullptr, T1, nullptr, 1.0 / 12.0, S, nullptr, -1.0), "G_a3");
        // G_W = -(1/60)[G_Y, a1] (T4); G_a1 += -(1/60)[W, G_Y]
        HIPCHK(gemm(Wn, A2, nullptr, Pl, nullptr, Em, nullptr, 1.0), "a1 G_Y");
        HIPCHK(gemm(Wn, Pl, nullptr, A2, nullptr, T4, nullptr, -1.0 / 60.0, Em, nullptr, 1.0 / 60.0), "G_W");
        HIPCHK(gemm(Wn, T2, nullptr, Pl, nullptr, Em, nullptr, 1.0), "W G_Y");
        HIPCHK(gemm(Wn, Pl, nullptr, T2, nullptr, A, nullptr, 1.0 / 60.0, Em, nullptr, -1.0 / 60.0), "[W, G_Y]");
        HIPCHK(axpby(Wn, A, nullptr, Qi, nullptr, 1.0, Qi, nullptr, 1.0), "G_a1 +");
        // G_a3 += 2 G_W; G_C1 = G_X + G_W (S)
        HIPCHK(axpby(Wn, T4, nullptr, T1, nullptr, 2.0, T1, nullptr, 1.0), "G_a3 +");
        HIPCHK(axpby(Wn, T4, nullptr, S, nullptr, 1.0, S, nullptr, 1.0), "G_C1");
        // G_a1 += [a2, G_C1]; G_a2 = G_Y + [G_C1, a1] (Pl)
        HIPCHK(gemm(Wn, R0, nullptr, S, nullptr, Em, nullptr, 1.0), "a2 G_C1");
        HIPCHK(gemm(Wn, S, nullptr, R0, nullptr, A, nullptr, -1.0, Em, nullptr, 1.0), "[a2, G_C1]");
        HIPCHK(axpby(Wn, A, nullptr, Qi, nullptr, 1.0, Qi, nullptr, 1.0), "G_a1 +");
        HIPCHK(gemm(Wn, S, nullptr, A2, nullptr, Em, nullptr, 1.0), "G_C1 a1");
        HIPCHK(gemm(Wn, A2, nullptr, S, nullptr, A, nullptr, -1.0, Em, nullptr, 1.0), "[G_C1, a1]");
        HIPCHK(axpby(Wn, A, nullptr, Pl, nullptr, 1.0, Pl, nullptr, 1.0), "G_a2");
      }
      {
        StageTimer t(c, 6, s);
        void* Ks[3] = {T3, nullptr, nullptr};
        if (c->order == 6) { Ks[0] = Qi; Ks[1] = Pl; Ks[2] = T1; }
        for (int pl = 0; pl < (c->order == 6 ? 3 : 1); ++pl) {
          BigTraceArgs ta{};
          ta.n = n; ta.n_slices = Wn; ta.nb = c->nb; ta.first_slice = w.s0; ta.trans_basis = 1;
          ta.K = Ks[pl]; ta.basis = c->basis32; ta.part = (double*)at(BL.part);
          ta.tile_ptr = c->tile_ptr; ta.tile_j = c->tile_j;
          ta.gtrace = (double*)at(BL.gtrace) + pl * coef_plane;
          HIPCHK(c->real ? launch_rtraces(ta, s) : launch_btraces(32, ta, s), "traces");
        }
      }
    }
  }
  if (grad || grouped) {
    GradArgs ga{};
    ga.prec = 32; ga.gtrace = grad ? (const double*)at(BL.gtrace) : nullptr;
    ga.amps = b->amps; ga.item_amp_offset = (const int64_t*)at(L.amp_off); ga.items = items;
    ga.n_items = (int)p.items.size(); ga.static_coef = b->static_coef; ga.ctrl_scale = b->ctrl_scale;
    ga.n_ctrl = c->nc; ga.n_static = c->ns; ga.order = c->order; ga.hold_foh = c->hold == LMAG_FOH;
    ga.nb = c->nb; ga.dt = b->dt; ga.inv_d2 = 1.0 / ((double)c->d * c->d);
    ga.n_slices_total = Ns;
    ga.grad = grad ? grad_out : nullptr;
    ga.group_first_item = grouped ? (const int32_t*)at(L.group_first) : nullptr;
    ga.group_items = grouped ? (const int32_t*)at(L.group_items) : nullptr;
    ga.n_groups = p.n_groups; ga.F_items = F_items; ga.F_out = grouped ? F_out : nullptr;
    ga.group_global = grouped ? (const int32_t*)at(L.group_global) : nullptr;
    StageTimer t(c, 7, s);
    HIPCHK(launch_grad(ga, grad ? p.max_slices : 1, s), "grad");
  }
  finish_plan();
  return LMAG_OK;
}


// Splits the batch into waves that fit the workspace budget (groups stay
// whole). A wave whose stored per-slice tiles do not fit runs in recompute
// mode; a unit that does not fit even then is LMAG_E_NOMEM.
lmag_status run_waves_body(lmag_ctx* c, const lmag_batch* b, const int32_t* target_of_item,
                           int n_targets, bool grad, bool fidelity, const void* U_target,
                           double* F_out, void* grad_out, void* S_out, hipStream_t s);

// Every compute call shares the context's workspace (plan, coefficients, tiles,
// work counters). A call on a stream other than the previous call's first makes
// its stream wait, on the device, for the previous call's completion event; the
// host does not block. The event is recorded again at the end of the call.
lmag_status run_waves(lmag_ctx* c, const lmag_batch* b, const int32_t* target_of_item,
                      int n_targets, bool grad, bool fidelity, const void* U_target,
                      double* F_out, void* grad_out, void* S_out, hipStream_t s) {
  lmag_status st = validate_batch(c, b, target_of_item, fidelity ? n_targets : 1, grad);
  if (st != LMAG_OK) return st;
  if (c->call_pending && s != c->last_stream)
    HIPCHK(hipStreamWaitEvent(s, c->call_done, 0), "hipStreamWaitEvent");
  c->last_stream = s;
  c->call_total = 0;
  for (int i = 0; i < b->n_items; ++i) c->call_total += b->n_slices[i];
  st = run_waves_body(c, b, target_of_item, n_targets, grad, fidelity, U_target, F_out, grad_out,
                      S_out, s);
  c->call_total = 0;
  hipError_t e = hipEventRecord(c->call_done, s);
  if (e != hipSuccess && st == LMAG_OK) return c->hip_fail(e, "hipEventRecord");
  c->call_pending = true;
  return st;
}

lmag_status run_waves_body(lmag_ctx* c, const lmag_batch* b, const int32_t* target_of_item,
                           int n_targets, bool grad, bool fidelity, const void* U_target,
                           double* F_out, void* grad_out, void* S_out, hipStream_t s) {
  lmag_status st = LMAG_OK;
  if (c->tiled)
    return run_big(c, b, target_of_item, n_targets, grad, fidelity, U_target, F_out, grad_out, S_out, s);
  // units: whole groups (grouped calls) or single items, in order
  std::vector<std::vector<int>> units;
  if (b->n_groups > 0) {
    units.resize(b->n_groups);
    for (int i = 0; i < b->n_items; ++i) units[b->group_of_item[i]].push_back(i);
  } else {
    units.resize(b->n_items);
    for (int i = 0; i < b->n_items; ++i) units[i].push_back(i);
  }
  const size_t budget = device_budget(c);
  const int nt = fidelity ? n_targets : 0;
  auto fits = [&](const std::vector<int>& idx, bool recompute, Plan& p, Layout& L, int& grid) {
    p = Plan();
    plan_wave(c, b, target_of_item, idx, p, recompute);
    p.recompute = recompute;
    grid = std::max(1, std::min(p.total_chunks, c->n_cu));
    L = layout(c, p, nt, grad, grid);
    if (recompute && L.total > budget) {
      // fewer persistent workgroups need less recompute scratch
      const size_t es = (c->prec == 32 ? 8 : 16);
      const size_t per_wg = (size_t)p.chunk_size * WS_TILES * TILE * es +
                            (c->prec == 64 ? (size_t)2 * SLOT * es : 0) + 512;
      const size_t over = L.total - budget;
      const int cut = (int)((over + per_wg - 1) / per_wg);
      if (cut >= grid) return false;
      grid -= cut;
      L = layout(c, p, nt, grad, grid);
      // the estimate ignores buffer alignment: drop workgroups until it fits
      while (L.total > budget && grid > 1) L = layout(c, p, nt, grad, --grid);
    }
    return L.total <= budget;
  };
  size_t u = 0;
  int waves = 0;
  while (u < units.size()) {
    std::vector<int> idx = units[u];
    Plan p;
    Layout L{};
    int grid = 0;
    bool recompute = false;
    if (!fits(idx, false, p, L, grid)) {
      if (!grad || !fits(idx, true, p, L, grid))
        return c->fail(LMAG_E_NOMEM, "one item (group) needs " + std::to_string(L.total) +
                                         " bytes of workspace, over the budget of " +
                                         std::to_string(budget));
      recompute = true;
    }
    size_t v = u + 1;
    if (!recompute) {
      // grow the wave by doubling, then by single units
      size_t step = 1;
      while (v < units.size()) {
        std::vector<int> trial = idx;
        const size_t end = std::min(units.size(), v + step);
        for (size_t k = v; k < end; ++k) trial.insert(trial.end(), units[k].begin(), units[k].end());
        Plan p2;
        Layout L2{};
        int g2 = 0;
        if (fits(trial, false, p2, L2, g2)) {
          idx.swap(trial);
          p = std::move(p2); L = L2; grid = g2;
          v = end;
          step *= 2;
        } else if (step > 1) {
          step = 1;
        } else {
          break;
        }
      }
    }
    st = ensure_ws(c, L.total);
    if (st != LMAG_OK) return st;
    st = upload_plan(c, p, L, s, c->ws);
    if (st != LMAG_OK) return st;
    c->plan_info[0] = p.total_slices;
    c->plan_info[1] = p.total_chunks;
    c->plan_info[2] = p.chunk_size;
    c->plan_info[3] = grid;
    c->plan_info[4] = (int64_t)L.total;
    c->plan_recompute = p.recompute;
    st = run(c, b, p, L, grad, fidelity, U_target, n_targets, F_out, grad_out, S_out, s, grid, c->ws);
    if (st != LMAG_OK) return st;
    u = v;
    ++waves;
  }
  c->plan_waves = waves;
  return LMAG_OK;
}

}  // namespace

extern "C" {

const char* lmag_version(void) { return "lmag 0.1 (gfx950)"; }

lmag_status lmag_create(lmag_ctx** out, int hip_device) {
  if (!out) return LMAG_E_INVALID;
  *out = nullptr;
  try {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) {
      (void)hipGetLastError();
      return LMAG_E_DEVICE;
    }
    lmag_ctx* c = new lmag_ctx();
    c->device = hip_device;
    DeviceGuard g(hip_device);
    if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess ||
        c->n_cu <= 0)
      c->n_cu = 256;
    if (hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->call_done, hipEventDisableTiming) != hipSuccess) {
      if (c->upload_done) (void)hipEventDestroy(c->upload_done);
      delete c;
      return LMAG_E_DEVICE;
    }
    c->scratch = scratch_address(c);   // checked again by the entry point that uses it
    pade_coeffs(3, c->pade.b3);
    pade_coeffs(5, c->pade.b5);
    pade_coeffs(7, c->pade.b7);
    pade_coeffs(2, c->pade.b2);
    c->pade.ser_max32_2 = series_limit32(c->pade.b2, 2, series_degree(2), true);
    c->pade.ser_max32_3 = series_limit32(c->pade.b3, 3, series_degree(3), false);
    pade_series(c->pade.b2, 2, c->pade.r2, 8);
    inv_series(c->pade.b3, 3, c->pade.c3, 8);
    *out = c;
    return LMAG_OK;
  } catch (...) {
    return LMAG_E_NOMEM;
  }
}

void lmag_destroy(lmag_ctx* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();
  if (c->ws) (void)hipFree(c->ws);
  if (c->basis64) (void)hipFree(c->basis64);
  if (c->basis32) (void)hipFree(c->basis32);
  if (c->sp_dev) (void)hipFree(c->sp_dev);
  if (c->tile_lists) (void)hipFree(c->tile_lists);
  if (c->logP_dev) (void)hipFree(c->logP_dev);
  if (c->dbg_scratch) (void)hipFree(c->dbg_scratch);
  if (c->clk_dev) (void)hipFree(c->clk_dev);
  if (c->mse_part) (void)hipFree(c->mse_part);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->upload_done) (void)hipEventDestroy(c->upload_done);
  if (c->call_done) (void)hipEventDestroy(c->call_done);
  for (auto& pe : c->ev_pending) { (void)hipEventDestroy(pe.second.first); (void)hipEventDestroy(pe.second.second); }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
}

const char* lmag_last_error(const lmag_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

static bool finite_array(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

lmag_status lmag_set_system(lmag_ctx* c, const lmag_system_desc* s) {
  if (!c) return LMAG_E_INVALID;
  try {
    if (!s) return c->fail(LMAG_E_INVALID, "system descriptor is NULL");
    const int d = s->d;
    if (d < 1 || d > 64) return c->fail(LMAG_E_INVALID, "d must satisfy 1 <= d <= 64");
    const bool big = d * d > 64 || s->magnus_order == 6;
    if (big && (d * d) % 64 != 0)
      return c->fail(LMAG_E_UNSUPPORTED, d * d > 64 ? "d*d must be <= 64 or a multiple of 64"
                                                    : "Magnus order 6 needs d*d a multiple of 64");
    if (big && s->precision != LMAG_F32)
      return c->fail(LMAG_E_UNSUPPORTED, "superoperators larger than 64 x 64 and Magnus order 6 run in FP32 only");
    if (s->n_static < 0 || s->n_ctrl < 0 || s->n_jump < 0)
      return c->fail(LMAG_E_INVALID, "negative operator count");
    if (s->n_ctrl > 8 || s->n_static > 8) return c->fail(LMAG_E_UNSUPPORTED, "at most 8 controls and 8 static terms");
    if ((s->n_static && !s->H_static) || (s->n_ctrl && !s->H_ctrl) || (s->n_jump && !s->L_jump))
      return c->fail(LMAG_E_INVALID, "operator array is NULL");
    if (s->precision != LMAG_F32 && s->precision != LMAG_F64)
      return c->fail(LMAG_E_INVALID, "precision must be LMAG_F32 or LMAG_F64");
    if (s->magnus_order != 1 && s->magnus_order != 2 && s->magnus_order != 6)
      return c->fail(LMAG_E_INVALID, "magnus_order must be 1, 2 or 6");
    if (s->hold != LMAG_ZOH && s->hold != LMAG_FOH) return c->fail(LMAG_E_INVALID, "hold must be ZOH or FOH");
    if (s->chunk_slices < 0) return c->fail(LMAG_E_INVALID, "chunk_slices < 0");
    if (s->basis != 0 && s->basis != 1)
      return c->fail(LMAG_E_INVALID, "basis must be 0 (Hermitian-operator basis) or 1 (column stacking)");
    const bool real = s->basis == 0 && s->precision == 32;
    const bool rbig = real && big;   // real FP32 matrices; the 64 x 64 tiles stay complex
    const size_t dd2 = (size_t)d * d * 2;
    if ((s->n_static && !finite_array(s->H_static, s->n_static * dd2)) ||
        (s->n_ctrl && !finite_array(s->H_ctrl, s->n_ctrl * dd2)) ||
        (s->n_jump && !finite_array(s->L_jump, s->n_jump * dd2)))
      return c->fail(LMAG_E_INVALID, "non-finite operator entry");
    const int nc = s->n_ctrl, ns = s->n_static;
    int nb = nc + ns + 1;
    if (s->magnus_order == 2) nb += nc + nc * ns + nc * (nc - 1) / 2;
    if (nb > (d * d > 64 ? MAX_BIG_NB : 32)) return c->fail(LMAG_E_UNSUPPORTED, "basis too large");

    DeviceGuard g(c->device);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return c->hip_fail(e, "hipDeviceSynchronize");
    if (c->basis64) (void)hipFree(c->basis64);
    if (c->basis32) (void)hipFree(c->basis32);
    if (c->sp_dev) (void)hipFree(c->sp_dev);
    if (c->tile_lists) (void)hipFree(c->tile_lists);
    c->basis64 = nullptr;
    c->basis32 = nullptr;
    c->sp_dev = nullptr;
    c->tile_lists = nullptr;
    c->tile_ptr = nullptr;
    c->tile_j = nullptr;
    c->sp = SparseBasis{};
    c->has_sys = false;
    const size_t nn = big ? (size_t)d * d * d * d : (size_t)TILE;   // elements per basis matrix
    const size_t tb = nn * 16;
    double* ops = nullptr;
    double* ldl = nullptr;
    double* tmp = nullptr;
    const size_t nops = (size_t)(ns + nc + s->n_jump) * dd2;
    if (hipMalloc((void**)&c->basis64, nb * tb) != hipSuccess ||
        hipMalloc(&c->basis32, nb * nn * (rbig ? 4 : 8)) != hipSuccess ||
        hipMalloc((void**)&ops, std::max<size_t>(8, nops * 8)) != hipSuccess ||
        hipMalloc((void**)&ldl, std::max<size_t>(8, (size_t)s->n_jump * dd2 * 8)) != hipSuccess ||
        (big && hipMalloc((void**)&tmp, tb) != hipSuccess)) {
      (void)hipGetLastError();
      if (ops) (void)hipFree(ops);
      if (ldl) (void)hipFree(ldl);
      if (tmp) (void)hipFree(tmp);
      return c->fail(LMAG_E_NOMEM, "basis allocation failed");
    }
    std::vector<double> hops(std::max<size_t>(1, nops));
    size_t o = 0;
    if (ns) std::memcpy(&hops[o], s->H_static, ns * dd2 * 8), o += ns * dd2;
    if (nc) std::memcpy(&hops[o], s->H_ctrl, nc * dd2 * 8), o += nc * dd2;
    if (s->n_jump) std::memcpy(&hops[o], s->L_jump, s->n_jump * dd2 * 8), o += s->n_jump * dd2;
    hipStream_t st = nullptr;
    if (nops) HIPCHK(hipMemcpy(ops, hops.data(), nops * 8, hipMemcpyHostToDevice), "hipMemcpy(ops)");
    const double* Hs = ops;
    const double* Hc = ops + ns * dd2;
    const double* Lj = ops + (ns + nc) * dd2;
    auto tile = [&](int j) { return c->basis64 + (size_t)j * nn * 2; };
    auto lift = [&](const double* H, double* out) {
      return big ? launch_blift(H, d, out, st) : launch_lift(H, d, out, st);
    };
    // [X, Y] = X Y - Y X: tile kernel for 64 x 64, two batched products otherwise
    auto comm = [&](const double* X, const double* Y, double* out) -> hipError_t {
      if (!big) return launch_commutator(X, Y, out, st);
      BigGemmArgs g{};
      g.n = d * d; g.batch = 1; g.A = X; g.B = Y; g.C = tmp; g.alpha = 1.0;
      hipError_t e = launch_bgemm(64, g, st);
      if (e != hipSuccess) return e;
      g.A = Y; g.B = X; g.C = out; g.D = tmp; g.alpha = -1.0; g.beta = 1.0;
      return launch_bgemm(64, g, st);
    };
    // L_c | Z_i | D | [L_c, D] | [L_c, Z_i] | [L_p, L_q]
    for (int cc = 0; cc < nc; ++cc) HIPCHK(lift(Hc + cc * dd2, tile(cc)), "lift");
    for (int i = 0; i < ns; ++i) HIPCHK(lift(Hs + i * dd2, tile(nc + i)), "lift");
    if (big) HIPCHK(launch_bdissipator(Lj, s->n_jump, d, ldl, tile(nc + ns), st), "dissipator");
    else HIPCHK(launch_dissipator(Lj, s->n_jump, d, tile(nc + ns), st), "dissipator");
    if (s->magnus_order == 2) {
      int j = nc + ns + 1;
      for (int cc = 0; cc < nc; ++cc) HIPCHK(comm(tile(cc), tile(nc + ns), tile(j++)), "comm");
      for (int cc = 0; cc < nc; ++cc)
        for (int i = 0; i < ns; ++i) HIPCHK(comm(tile(cc), tile(nc + i), tile(j++)), "comm");
      for (int p = 0; p < nc; ++p)
        for (int q = p + 1; q < nc; ++q) HIPCHK(comm(tile(p), tile(q), tile(j++)), "comm");
    }
    if (rbig) {
      // the real form R_j = T B_j T^dag in the basis of Hermitian operators,
      // kept in FP64 for the tile lists and cast to the FP32 copy
      double* r64 = nullptr;
      if (hipMalloc((void**)&r64, (size_t)nb * nn * 8) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(ops);
        (void)hipFree(ldl);
        if (tmp) (void)hipFree(tmp);
        return c->fail(LMAG_E_NOMEM, "basis allocation failed");
      }
      HIPCHK(launch_to_real(c->basis64, d, nb, r64, st), "basis (real)");
      HIPCHK(launch_rcast(r64, (float*)c->basis32, (size_t)nb * nn, st), "cast");
      HIPCHK(hipDeviceSynchronize(), "set_system sync");
      (void)hipFree(c->basis64);
      c->basis64 = r64;
    } else {
      // 64 x 64 tiles in the real basis: (R_j, 0) in place, in FP64 for the
      // sparse-support analysis below
      if (real) HIPCHK(launch_tile_to_real(c->basis64, nb, d, nullptr, st), "basis (real)");
      HIPCHK(launch_cast(c->basis64, (float*)c->basis32, (size_t)nb * nn * 2, st), "cast");
      HIPCHK(hipDeviceSynchronize(), "set_system sync");
    }
    if (big) {
      // the basis elements with a nonzero 64 x 64 tile, per tile position:
      // the exponent assembly and the traces skip the all-zero tiles
      const int Tn = d * d / 64;
      const size_t nt = (size_t)Tn * Tn;
      uint8_t* fl = nullptr;
      std::vector<uint8_t> flh((size_t)nb * nt);
      if (hipMalloc((void**)&fl, flh.size()) == hipSuccess) {
        if ((rbig ? launch_rtile_flags(c->basis64, nb, d * d, fl, st)
                  : launch_tile_flags(c->basis64, nb, d * d, fl, st)) == hipSuccess &&
            hipMemcpy(flh.data(), fl, flh.size(), hipMemcpyDeviceToHost) == hipSuccess) {
          std::vector<int32_t> lists(nt + 1, 0);
          for (size_t t = 0; t < nt; ++t)
            for (int j = 0; j < nb; ++j)
              if (flh[(size_t)j * nt + t]) lists.push_back(j);
          int32_t pos = (int32_t)(nt + 1);
          for (size_t t = 0; t < nt; ++t) {
            lists[t] = pos - (int32_t)(nt + 1);
            for (int j = 0; j < nb; ++j) pos += flh[(size_t)j * nt + t] ? 1 : 0;
          }
          lists[nt] = pos - (int32_t)(nt + 1);
          if (hipMalloc((void**)&c->tile_lists, lists.size() * 4) == hipSuccess &&
              hipMemcpy(c->tile_lists, lists.data(), lists.size() * 4, hipMemcpyHostToDevice) == hipSuccess) {
            c->tile_ptr = c->tile_lists;
            c->tile_j = c->tile_lists + nt + 1;
          } else {
            if (c->tile_lists) (void)hipFree(c->tile_lists);
            c->tile_lists = nullptr;
          }
        }
        (void)hipFree(fl);
      }
      (void)hipGetLastError();   // without the lists every tile is visited
      // the block-tiled path (FP32) reads only the FP32 copy
      (void)hipFree(c->basis64);
      c->basis64 = nullptr;
    }
    if (!big) {
      std::vector<double> hb((size_t)nb * TILE * 2);
      HIPCHK(hipMemcpy(hb.data(), c->basis64, hb.size() * 8, hipMemcpyDeviceToHost), "basis copy");
      build_sparse(c, hb, nb, s->precision);
    }
    (void)hipFree(ops);
    (void)hipFree(ldl);
    if (tmp) (void)hipFree(tmp);
    c->d = d; c->n = d * d; c->ns = ns; c->nc = nc; c->nj = s->n_jump;
    c->prec = s->precision; c->order = s->magnus_order; c->hold = s->hold; c->nb = nb;
    c->chunk = s->chunk_slices; c->ws_max = s->workspace_bytes_max;
    c->tiled = big;
    c->real = real;
    c->has_sys = true;
    return LMAG_OK;
  } catch (const std::bad_alloc&) {
    return c->fail(LMAG_E_NOMEM, "host allocation failed");
  } catch (const std::exception& ex) {
    return c->fail(LMAG_E_DEVICE, ex.what());
  } catch (...) {
    return c->fail(LMAG_E_DEVICE, "unknown error");
  }
}

lmag_status lmag_propagate(lmag_ctx* c, const lmag_batch* b, void* S_out, void* hip_stream) {
  if (!c) return LMAG_E_INVALID;
  try {
    if (!c->has_sys) return c->fail(LMAG_E_NOSYSTEM, "lmag_set_system has not been called");
    if (!S_out) return c->fail(LMAG_E_INVALID, "S_out is NULL");
    if (b && b->n_groups) return c->fail(LMAG_E_INVALID, "groups apply to fidelity calls only");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)hip_stream;
    return run_waves(c, b, nullptr, 0, false, false, nullptr, nullptr, nullptr, S_out, s);
  } catch (const std::bad_alloc&) {
    return c->fail(LMAG_E_NOMEM, "host allocation failed");
  } catch (...) {
    return c->fail(LMAG_E_DEVICE, "unknown error");
  }
}

lmag_status lmag_fidelity_and_grad(lmag_ctx* c, const lmag_batch* b, const void* U_target,
                                   int n_targets, const int32_t* target_of_item, double* F_out,
                                   void* grad_out, void* hip_stream) {
  if (!c) return LMAG_E_INVALID;
  try {
    if (!c->has_sys) return c->fail(LMAG_E_NOSYSTEM, "lmag_set_system has not been called");
    if (!U_target || n_targets < 1) return c->fail(LMAG_E_INVALID, "U_target NULL or n_targets < 1");
    if (!F_out) return c->fail(LMAG_E_INVALID, "F_out is NULL");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)hip_stream;
    return run_waves(c, b, target_of_item, n_targets, grad_out != nullptr, true, U_target, F_out,
                     grad_out, nullptr, s);
  } catch (const std::bad_alloc&) {
    return c->fail(LMAG_E_NOMEM, "host allocation failed");
  } catch (...) {
    return c->fail(LMAG_E_DEVICE, "unknown error");
  }
}

lmag_status lmag_fidelity_and_grad_noalloc(lmag_ctx* c, const lmag_batch* b, const void* U_target,
                                           int n_targets, const int32_t* target_of_item,
                                           double* F_out, void* grad_out, void* hip_stream) {
  if (!c) return LMAG_E_INVALID;
  try {
    if (!c->has_sys) return c->fail(LMAG_E_NOSYSTEM, "lmag_set_system has not been called");
    if (!U_target || n_targets < 1) return c->fail(LMAG_E_INVALID, "U_target NULL or n_targets < 1");
    if (!F_out) return c->fail(LMAG_E_INVALID, "F_out is NULL");
    if (c->tiled)
      return c->fail(LMAG_E_UNSUPPORTED, "the no-allocation entry point covers the 64 x 64 slice kernels "
                                         "(superoperators up to 64 x 64, Magnus order 1 or 2)");
    if (!c->scratch) return c->fail(LMAG_E_DEVICE, "no address for the scratch array on this device");
    const bool grad = grad_out != nullptr;
    lmag_status st = validate_batch(c, b, target_of_item, n_targets, grad);
    if (st != LMAG_OK) return st;
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)hip_stream;
    std::vector<int> all(b->n_items);
    for (int i = 0; i < b->n_items; ++i) all[i] = i;
    Plan p;
    plan_wave(c, b, target_of_item, all, p, false);
    p.recompute = false;
    const int grid = std::max(1, std::min(p.total_chunks, c->n_cu));
    const Layout L = layout(c, p, n_targets, grad, grid);
    if (L.total > kScratchBytes)
      return c->fail(LMAG_E_INVALID, "the call needs " + std::to_string(L.total) +
                                         " bytes of workspace, over the fixed scratch of " +
                                         std::to_string(kScratchBytes) +
                                         " bytes: split the batch, or use lmag_fidelity_and_grad");
    if (c->call_pending && s != c->last_stream)
      HIPCHK(hipStreamWaitEvent(s, c->call_done, 0), "hipStreamWaitEvent");
    c->last_stream = s;
    st = upload_plan(c, p, L, s, c->scratch, false);
    if (st == LMAG_OK) {
      c->plan_info[0] = p.total_slices; c->plan_info[1] = p.total_chunks;
      c->plan_info[2] = p.chunk_size; c->plan_info[3] = grid; c->plan_info[4] = (int64_t)L.total;
      c->plan_recompute = false;
      c->plan_waves = 1;
      st = run(c, b, p, L, grad, true, U_target, n_targets, F_out, grad_out, nullptr, s, grid,
               c->scratch);
    }
    const hipError_t e = hipEventRecord(c->call_done, s);
    if (e != hipSuccess && st == LMAG_OK) return c->hip_fail(e, "hipEventRecord");
    c->call_pending = true;
    return st;
  } catch (const std::bad_alloc&) {
    return c->fail(LMAG_E_NOMEM, "host allocation failed");
  } catch (...) {
    return c->fail(LMAG_E_DEVICE, "unknown error");
  }
}

lmag_status lmag_adam_project(lmag_ctx* c, int precision, int64_t rows, int n_ctrl, void* amps,
                              const void* grad, void* m_state, void* v_state, int step, double lr,
                              double beta1, double beta2, double eps, double grad_scale, double lo,
                              double hi, const uint8_t* row_active, void* hip_stream) {
  if (!c) return LMAG_E_INVALID;
  if (precision != LMAG_F32 && precision != LMAG_F64) return c->fail(LMAG_E_INVALID, "precision");
  if (rows < 0 || n_ctrl < 1) return c->fail(LMAG_E_INVALID, "rows < 0 or n_ctrl < 1");
  if (rows > 0 && (!amps || !grad || !m_state || !v_state)) return c->fail(LMAG_E_INVALID, "NULL array");
  if (step < 1) return c->fail(LMAG_E_INVALID, "step must be >= 1");
  if (!(lr >= 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0) ||
      !std::isfinite(grad_scale) || !(lo <= hi))
    return c->fail(LMAG_E_INVALID, "bad hyper-parameters");
  DeviceGuard g(c->device);
  AdamArgs a{};
  a.n = rows * (int64_t)n_ctrl; a.row_len = n_ctrl;
  a.theta = amps; a.grad = grad; a.m = m_state; a.v = v_state;
  a.lr = lr; a.beta1 = beta1; a.beta2 = beta2; a.eps = eps;
  a.bc1 = 1.0 - std::pow(beta1, (double)step); a.bc2 = 1.0 - std::pow(beta2, (double)step);
  a.grad_scale = grad_scale; a.lo = lo; a.hi = hi; a.row_active = row_active;
  HIPCHK(launch_adam_project(precision, a, (hipStream_t)hip_stream), "adam");
  return LMAG_OK;
}

lmag_status lmag_autotune(lmag_ctx* c, const lmag_batch* b, const void* U_target, int n_targets,
                          const int32_t* target_of_item, int reps, int32_t* best_out,
                          double* best_ms_out, void* hip_stream) {
  if (!c) return LMAG_E_INVALID;
  try {
    if (!c->has_sys) return c->fail(LMAG_E_NOSYSTEM, "lmag_set_system has not been called");
    if (!U_target || n_targets < 1) return c->fail(LMAG_E_INVALID, "U_target NULL or n_targets < 1");
    if (reps < 1) return c->fail(LMAG_E_INVALID, "reps must be >= 1");
    lmag_status st = validate_batch(c, b, target_of_item, n_targets, true);
    if (st != LMAG_OK) return st;
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)hip_stream;
    long long total = 0;
    int64_t rows = 0;
    for (int i = 0; i < b->n_items; ++i) {
      total += b->n_slices[i];
      rows = std::max<int64_t>(rows, b->slice_offset[i] + b->n_slices[i]);
    }
    const size_t es = c->prec == 32 ? 4 : 8;
    void* Fd = nullptr;
    void* Gd = nullptr;
    const int nf = b->n_groups > 0 ? b->n_groups : b->n_items;
    if (hipMalloc(&Fd, (size_t)nf * 8) != hipSuccess ||
        hipMalloc(&Gd, std::max<size_t>(8, (size_t)rows * c->nc * es)) != hipSuccess) {
      (void)hipGetLastError();
      if (Fd) (void)hipFree(Fd);
      return c->fail(LMAG_E_NOMEM, "autotune output buffers");
    }
    const int saved_chunk = c->chunk, saved_inv = c->inv_variant, saved_big = c->big_variant;
    const bool big = c->tiled;
    const long long per = (total + c->n_cu - 1) / std::max(1, c->n_cu);
    std::vector<int> chunks;
    if (big) {
      // block-tiled path: the product kernel (tile ownership and MFMA shape) at
      // the automatic chunk length and at half and twice it
      const int C0 = big_auto_chunk(c, total);
      for (int C : {C0, std::max(1, C0 / 2), 2 * C0})
        if (std::find(chunks.begin(), chunks.end(), C) == chunks.end()) chunks.push_back(C);
    } else {
      for (int C : {2, 4, 8, 16, 32, 64, 128, 256})
        if (C <= std::max<long long>(2, 4 * per) && C >= std::min<long long>(per / 4, 64)) chunks.push_back(C);
      if (chunks.empty()) chunks.push_back(auto_chunk(c, total, false));
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    double best = 1e300;
    int bestC = chunks[0], bestInv = 0;
    std::vector<int> variants{0, 1, 2};
    if (big && c->real) {
      // the real product kernels: 64 x 64 tiles without and with the next
      // k-step's tiles requested ahead, each without and with the XCD
      // grouping; 128 x 128 tiles
      variants = {0, 2};
      if ((c->n / 64) % 2 == 0) variants.push_back(1);
      if (c->n / 64 <= 16) {
        variants.push_back(5);
        variants.push_back(7);
      }
    } else if (big) {
      variants.push_back(3);
      if ((c->n / 64) % 2 == 0) variants.push_back(4);
      variants.push_back(6);
      variants.push_back(8);
      if (c->n / 64 <= 16) {
        variants.push_back(5);
        variants.push_back(7);
      }
    }
    for (int inv : variants) {
      for (int C : chunks) {
        c->chunk = C;
        if (big) c->big_variant = inv;
        else c->inv_variant = inv;
        st = run_waves(c, b, target_of_item, n_targets, true, true, U_target, (double*)Fd, Gd,
                       nullptr, s);   // warm-up (also sizes the workspace)
        if (st != LMAG_OK) break;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps && st == LMAG_OK; ++r)
          st = run_waves(c, b, target_of_item, n_targets, true, true, U_target, (double*)Fd, Gd,
                         nullptr, s);
        (void)hipEventRecord(e1, s);
        if (st != LMAG_OK) break;
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          st = c->hip_fail(hipGetLastError(), "autotune timing");
          break;
        }
        const double per_call = ms / reps;
        if (per_call < best) { best = per_call; bestC = C; bestInv = inv; }
        if (std::getenv("LMAG_TUNE_VERBOSE")) {
          std::fprintf(stderr, "lmag_autotune: variant %d chunk %d: %.4f ms per call\n", inv, C, per_call);
          std::fflush(stderr);
        }
      }
      if (st != LMAG_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(Fd);
    (void)hipFree(Gd);
    c->chunk = saved_chunk;
    c->inv_variant = saved_inv;
    c->big_variant = saved_big;
    if (st != LMAG_OK) return st;
    const std::string k = tune_key(c, total);
    bool found = false;
    for (auto& t : c->tuned)
      if (t.first == k) { t.second = {bestC, bestInv}; found = true; }
    if (!found) c->tuned.push_back({k, {bestC, bestInv}});
    if (const char* path = std::getenv("LMAG_TUNE_CACHE")) {
      if (FILE* f = std::fopen(path, "a")) {
        std::fprintf(f, "{\"key\": \"%s\", \"chunk\": %d, \"variant\": %d, \"ms\": %.4f}\n",
                     k.c_str(), bestC, bestInv, best);
        std::fclose(f);
      }
    }
    if (best_out) { best_out[0] = bestC; best_out[1] = bestInv; }
    if (best_ms_out) *best_ms_out = best;
    return LMAG_OK;
  } catch (const std::bad_alloc&) {
    return c->fail(LMAG_E_NOMEM, "host allocation failed");
  } catch (...) {
    return c->fail(LMAG_E_DEVICE, "unknown error");
  }
}

lmag_status lmag_load_tuning(lmag_ctx* c, const char* path) {
  if (!c) return LMAG_E_INVALID;
  if (!path) return c->fail(LMAG_E_INVALID, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return c->fail(LMAG_E_INVALID, std::string("cannot open ") + path);
  char line[512];
  int n = 0;
  while (std::fgets(line, sizeof(line), f)) {
    char key[128];
    int C = 0, inv = 0;
    if ((std::sscanf(line, " {\"key\": \"%127[^\"]\", \"chunk\": %d, \"variant\": %d", key, &C, &inv) == 3 ||
         std::sscanf(line, " {\"key\": \"%127[^\"]\", \"chunk\": %d, \"inverse\": %d", key, &C, &inv) == 3) &&
        C > 0 && inv >= 0 && inv < kBigGemmVariants) {
      bool found = false;
      for (auto& t : c->tuned)
        if (t.first == key) { t.second = {C, inv}; found = true; }
      if (!found) c->tuned.push_back({key, {C, inv}});
      ++n;
    }
  }
  std::fclose(f);
  return LMAG_OK;
}

lmag_status lmag_mlp_forward(lmag_ctx* c, int rows, int n_in, int n_out, const uint16_t* X,
                             const uint16_t* W, const float* b, int act, float scale, float* pre_out,
                             void* Y, void* hip_stream) {
  if (!c) return LMAG_E_INVALID;
  if (rows < 0 || n_in < 1 || n_out < 1) return c->fail(LMAG_E_INVALID, "bad layer shape");
  if (rows > 0 && (!X || !W || !b || !Y)) return c->fail(LMAG_E_INVALID, "NULL array");
  if (act != LMAG_ACT_GELU && act != LMAG_ACT_SIGMOID) return c->fail(LMAG_E_INVALID, "act");
  DeviceGuard g(c->device);
  MlpGemmArgs a{};
  a.M = rows; a.N = n_out; a.K = n_in;
  a.A = X; a.lda_r = n_in; a.lda_c = 1;
  a.B = W; a.ldb_r = 1; a.ldb_c = n_in;      // B(k, j) = W[j][k]
  a.bias = b; a.scale = scale; a.C32 = pre_out;
  if (act == LMAG_ACT_GELU) { a.mode = MLP_BIAS_GELU; a.C16 = (uint16_t*)Y; }
  else { a.mode = MLP_BIAS_SIGMOID; a.Y32 = (float*)Y; }
  HIPCHK(launch_mlp_gemm(a, (hipStream_t)hip_stream), "mlp_forward");
  return LMAG_OK;
}

lmag_status lmag_mlp_backward(lmag_ctx* c, int rows, int n_in, int n_out, const uint16_t* X,
                              const uint16_t* W, const uint16_t* G16, const float* G32, float* dW,
                              float* db, const float* pre_prev, uint16_t* dprev16, float* dprev32,
                              void* hip_stream) {
  if (!c) return LMAG_E_INVALID;
  if (rows < 1 || n_in < 1 || n_out < 1) return c->fail(LMAG_E_INVALID, "bad layer shape");
  if (!X || !W || !G16 || !G32 || !dW || !db) return c->fail(LMAG_E_INVALID, "NULL array");
  if (dprev16 && !pre_prev) return c->fail(LMAG_E_INVALID, "pre_prev NULL");
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)hip_stream;
  MlpGemmArgs a{};
  // dW[j][k] = sum_i G[i][j] X[i][k]
  a.M = n_out; a.N = n_in; a.K = rows;
  a.A = G16; a.lda_r = 1; a.lda_c = n_out;
  a.B = X; a.ldb_r = n_in; a.ldb_c = 1;
  a.mode = MLP_STORE; a.C32 = dW;
  HIPCHK(launch_mlp_gemm(a, s), "mlp_dW");
  HIPCHK(launch_colsum(G32, rows, n_out, db, s), "mlp_db");
  if (dprev16) {
    MlpGemmArgs d{};
    // dX[i][k] = sum_j G[i][j] W[j][k], times gelu'(pre_prev[i][k])
    d.M = rows; d.N = n_in; d.K = n_out;
    d.A = G16; d.lda_r = n_out; d.lda_c = 1;
    d.B = W; d.ldb_r = n_in; d.ldb_c = 1;
    d.mode = MLP_GELU_GRAD; d.aux = pre_prev; d.C16 = dprev16; d.C32 = dprev32;
    HIPCHK(launch_mlp_gemm(d, s), "mlp_dX");
  }
  return LMAG_OK;
}

lmag_status lmag_mlp_mse(lmag_ctx* c, int64_t n, const float* z, const float* y, float* dz32,
                         uint16_t* dz16, double* loss, void* hip_stream) {
  if (!c) return LMAG_E_INVALID;
  if (n < 1 || !z || !y || !loss) return c->fail(LMAG_E_INVALID, "bad MSE arguments");
  DeviceGuard g(c->device);
  if (!c->mse_part) {
    if (hipMalloc((void**)&c->mse_part, 256 * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      c->mse_part = nullptr;
      return c->fail(LMAG_E_NOMEM, "mse scratch");
    }
  }
  HIPCHK(launch_mse(z, y, n, dz32, dz16, c->mse_part, loss, (hipStream_t)hip_stream), "mlp_mse");
  return LMAG_OK;
}

lmag_status lmag_cast_bf16(lmag_ctx* c, const float* in, uint16_t* out, int64_t n, void* hip_stream) {
  if (!c) return LMAG_E_INVALID;
  if (n < 0 || (n > 0 && (!in || !out))) return c->fail(LMAG_E_INVALID, "bad cast arguments");
  DeviceGuard g(c->device);
  HIPCHK(launch_cast_bf16(in, out, n, (hipStream_t)hip_stream), "cast_bf16");
  return LMAG_OK;
}

lmag_status lmag_logical_score_and_grad(lmag_ctx* c, const lmag_batch* b, int kind, int L,
                                        const double* P, const void* T, int n_targets,
                                        const int32_t* target_of_item, double* score_out,
                                        void* grad_out, void* hip_stream) {
  if (!c) return LMAG_E_INVALID;
  try {
    if (!c->has_sys) return c->fail(LMAG_E_NOSYSTEM, "lmag_set_system has not been called");
    if (kind != LMAG_SCORE_PROJECTED && kind != LMAG_SCORE_LINEAR)
      return c->fail(LMAG_E_INVALID, "unknown score kind");
    if (L < 1 || L > MAX_LOGICAL) return c->fail(LMAG_E_INVALID, "L must be 1..4");
    if (!P || !T || n_targets < 1) return c->fail(LMAG_E_INVALID, "P or T NULL, or n_targets < 1");
    if (!score_out) return c->fail(LMAG_E_INVALID, "score_out is NULL");
    if (c->tiled) return c->fail(LMAG_E_UNSUPPORTED, "logical scores need d * d <= 64 and Magnus order 1 or 2");
    if (!finite_array(P, (size_t)c->n * L * 2)) return c->fail(LMAG_E_INVALID, "non-finite P");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)hip_stream;
    if (!c->logP_dev) {
      hipError_t e = hipMalloc((void**)&c->logP_dev, (size_t)64 * MAX_LOGICAL * 16);
      if (e != hipSuccess) { c->logP_dev = nullptr; return c->hip_fail(e, "hipMalloc(P)"); }
    }
    // P arrives column by column (n x L); the kernel reads [64][L] rows, zero padded
    std::vector<double> h((size_t)64 * L * 2, 0.0);
    for (int k = 0; k < L; ++k)
      for (int i = 0; i < c->n; ++i) {
        h[((size_t)i * L + k) * 2] = P[((size_t)k * c->n + i) * 2];
        h[((size_t)i * L + k) * 2 + 1] = P[((size_t)k * c->n + i) * 2 + 1];
      }
    if (c->real) {
      // in the basis of Hermitian operators the score reads T P: with
      // U = T^dag R T, P^dag U P = (T P)^dag R (T P). Row a = k + l d of T
      // has T[a][a] = 1 (k = l), 1/sqrt 2 (k < l) or i/sqrt 2 (k > l), and
      // T[a][l + k d] = 1/sqrt 2 (k < l) or -i/sqrt 2 (k > l).
      const double r = std::sqrt(0.5);
      std::vector<double> t(h.size(), 0.0);
      const int d = c->d;
      for (int a = 0; a < c->n; ++a) {
        const int kk = a % d, ll = a / d, q = ll + kk * d;
        for (int k = 0; k < L; ++k) {
          const double* x = &h[((size_t)a * L + k) * 2];
          const double* y = &h[((size_t)q * L + k) * 2];
          double* o = &t[((size_t)a * L + k) * 2];
          if (kk == ll) { o[0] = x[0]; o[1] = x[1]; }
          else if (kk < ll) { o[0] = r * (x[0] + y[0]); o[1] = r * (x[1] + y[1]); }
          else { o[0] = r * (y[1] - x[1]); o[1] = r * (x[0] - y[0]); }   // i r x - i r y
        }
      }
      h.swap(t);
    }
    HIPCHK(hipMemcpyAsync(c->logP_dev, h.data(), h.size() * 8, hipMemcpyHostToDevice, s), "P upload");
    HIPCHK(hipStreamSynchronize(s), "P upload");
    c->score_kind = kind;
    c->score_L = L;
    const lmag_status st = run_waves(c, b, target_of_item, n_targets, grad_out != nullptr, true, T,
                                     score_out, grad_out, nullptr, s);
    c->score_kind = 0;
    c->score_L = 0;
    return st;
  } catch (const std::bad_alloc&) {
    c->score_kind = 0;
    return c->fail(LMAG_E_NOMEM, "host allocation failed");
  } catch (...) {
    c->score_kind = 0;
    return c->fail(LMAG_E_DEVICE, "unknown error");
  }
}

lmag_status lmag_sync(lmag_ctx* c, void* hip_stream) {
  if (!c) return LMAG_E_INVALID;
  DeviceGuard g(c->device);
  hipError_t e = hipStreamSynchronize((hipStream_t)hip_stream);
  if (e != hipSuccess) return c->hip_fail(e, "hipStreamSynchronize");
  e = hipGetLastError();
  if (e != hipSuccess) return c->hip_fail(e, "pending device error");
  return LMAG_OK;
}

lmag_status lmag_pade_coefficients(int m, double* b_out) {
  if (!b_out || (m != 2 && m != 3 && m != 5 && m != 7)) return LMAG_E_INVALID;
  pade_coeffs(m, b_out);
  return LMAG_OK;
}

lmag_status lmag_pade_theta(int precision, int m, double* theta_out) {
  if (!theta_out) return LMAG_E_INVALID;
  if (precision == LMAG_F32) {
    if (m != 2 && m != 3) return LMAG_E_INVALID;
    *theta_out = m == 2 ? kTheta32_2 : kTheta32_3;
    return LMAG_OK;
  }
  if (precision == LMAG_F64) {
    if (m == 3) *theta_out = kTheta64[0];
    else if (m == 5) *theta_out = kTheta64[1];
    else if (m == 7) *theta_out = kTheta64[2];
    else return LMAG_E_INVALID;
    return LMAG_OK;
  }
  return LMAG_E_INVALID;
}

lmag_status lmag_last_selection_histogram(lmag_ctx* c, int64_t* counts) {
  if (!c) return LMAG_E_INVALID;
  if (!counts) return c->fail(LMAG_E_INVALID, "counts is NULL");
  DeviceGuard g(c->device);
  std::memset(counts, 0, sizeof(int64_t) * 4 * 64);
  if (!c->last_ms || c->last_total_slices <= 0) return LMAG_OK;
  std::vector<int8_t> h((size_t)c->last_total_slices * 2);
  hipError_t e = hipStreamSynchronize(c->last_stream);
  if (e != hipSuccess) return c->hip_fail(e, "hipStreamSynchronize");
  e = hipMemcpy(h.data(), c->last_ms, h.size(), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return c->hip_fail(e, "hipMemcpy(ms)");
  for (int i = 0; i < c->last_total_slices; ++i) {
    const int m = h[2 * i], s = h[2 * i + 1];
    const int mi = m == 2 ? 0 : (m == 3 ? 1 : (m == 5 ? 2 : (m == 7 ? 3 : -1)));
    if (mi >= 0 && s >= 0 && s < 64) counts[mi * 64 + s]++;
  }
  return LMAG_OK;
}

lmag_status lmag_set_profiling(lmag_ctx* c, int enable) {
  if (!c) return LMAG_E_INVALID;
  c->prof = enable != 0;
  return LMAG_OK;
}

lmag_status lmag_read_profile(lmag_ctx* c, double* ms, int64_t* cnt) {
  if (!c) return LMAG_E_INVALID;
  if (!ms || !cnt) return c->fail(LMAG_E_INVALID, "NULL output");
  DeviceGuard g(c->device);
  for (int i = 0; i < LMAG_STAGES; ++i) { ms[i] = 0.0; cnt[i] = 0; }
  lmag_status st = LMAG_OK;
  for (auto& pe : c->ev_pending) {
    hipEvent_t a = pe.second.first, b = pe.second.second;
    if (st == LMAG_OK) {
      hipError_t e = hipEventSynchronize(b);
      float t = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
      if (e != hipSuccess) st = c->hip_fail(e, "hipEventElapsedTime");
      else if (pe.first >= 0 && pe.first < LMAG_STAGES) { ms[pe.first] += t; cnt[pe.first] += 1; }
    }
    c->ev_pool.push_back(a);
    c->ev_pool.push_back(b);
  }
  c->ev_pending.clear();
  return st;
}

lmag_status lmag_debug_phase_cycles(lmag_ctx* c, int enable, int64_t* out) {
  if (!c) return LMAG_E_INVALID;
  DeviceGuard g(c->device);
  if (enable >= 0) {
    if (enable && !c->clk_dev) {
      hipError_t e = hipMalloc((void**)&c->clk_dev, 32 * sizeof(long long));
      if (e != hipSuccess) { (void)hipGetLastError(); c->clk_dev = nullptr; return c->fail(LMAG_E_NOMEM, "clock buffer"); }
    }
    if (enable) {
      HIPCHK(hipDeviceSynchronize(), "sync");
      HIPCHK(hipMemset(c->clk_dev, 0, 32 * sizeof(long long)), "memset");
    }
    c->clk_on = enable != 0;
  }
  if (out) {
    for (int i = 0; i < 32; ++i) out[i] = 0;
    if (c->clk_dev) {
      HIPCHK(hipDeviceSynchronize(), "sync");
      long long h[32];
      HIPCHK(hipMemcpy(h, c->clk_dev, sizeof(h), hipMemcpyDeviceToHost), "memcpy");
      for (int i = 0; i < 32; ++i) out[i] = h[i];
    }
  }
  return LMAG_OK;
}

lmag_status lmag_last_plan(lmag_ctx* c, int64_t* out) {
  if (!c) return LMAG_E_INVALID;
  if (!out) return c->fail(LMAG_E_INVALID, "NULL output");
  for (int i = 0; i < 5; ++i) out[i] = c->plan_info[i];
  out[5] = c->plan_recompute ? 1 : 0;
  out[6] = c->plan_waves;
  out[7] = c->sp.n_sup;
  return LMAG_OK;
}

lmag_status lmag_debug_tile_gemm(lmag_ctx* c, int precision, const void* A, const void* B, void* C,
                                 int transA, void* hip_stream) {
  if (!c) return LMAG_E_INVALID;
  if (!A || !B || !C) return c->fail(LMAG_E_INVALID, "NULL tile");
  if (precision != LMAG_F32 && precision != LMAG_F64) return c->fail(LMAG_E_INVALID, "precision");
  DeviceGuard g(c->device);
  HIPCHK(launch_debug_gemm(precision, A, B, C, transA, (hipStream_t)hip_stream), "debug_gemm");
  return LMAG_OK;
}

lmag_status lmag_debug_block_gemm(lmag_ctx* c, int n, int batch, const void* A, const void* B, void* C,
                                  int variant, void* hip_stream) {
  if (!c) return LMAG_E_INVALID;
  if (!A || !B || !C) return c->fail(LMAG_E_INVALID, "NULL matrix");
  if (n < 64 || n > 4096 || n % 64 != 0) return c->fail(LMAG_E_INVALID, "n must be a multiple of 64 in [64, 4096]");
  if (batch < 0) return c->fail(LMAG_E_INVALID, "batch < 0");
  if (variant < 0 || variant >= kBigGemmVariants) return c->fail(LMAG_E_INVALID, "product kernel variant");
  if (C == A || C == B) return c->fail(LMAG_E_INVALID, "C must not alias A or B");
  DeviceGuard g(c->device);
  BigGemmArgs a{};
  a.n = n; a.batch = batch; a.A = A; a.B = B; a.C = C; a.alpha = 1.0; a.variant = variant;
  HIPCHK(launch_bgemm(32, a, (hipStream_t)hip_stream), "debug block gemm");
  return LMAG_OK;
}

lmag_status lmag_debug_tile_inverse(lmag_ctx* c, int precision, const void* A, void* C, void* hip_stream) {
  if (!c) return LMAG_E_INVALID;
  if (!A || !C) return c->fail(LMAG_E_INVALID, "NULL tile");
  if (precision != LMAG_F32 && precision != LMAG_F64) return c->fail(LMAG_E_INVALID, "precision");
  DeviceGuard g(c->device);
  HIPCHK(launch_debug_inverse(precision, A, C, (hipStream_t)hip_stream), "debug_inverse");
  return LMAG_OK;
}

lmag_status lmag_debug_tile_expm(lmag_ctx* c, int precision, const void* A, void* C, int8_t* ms,
                                 void* hip_stream) {
  if (!c) return LMAG_E_INVALID;
  if (!A || !C || !ms) return c->fail(LMAG_E_INVALID, "NULL pointer");
  if (precision != LMAG_F32 && precision != LMAG_F64) return c->fail(LMAG_E_INVALID, "precision");
  DeviceGuard g(c->device);
  if (!c->dbg_scratch) {
    hipError_t e = hipMalloc(&c->dbg_scratch, (size_t)4 * SLOT * 16);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      c->dbg_scratch = nullptr;
      return c->fail(LMAG_E_NOMEM, "debug scratch");
    }
  }
  HIPCHK(launch_debug_expm(precision, A, C, ms, c->dbg_scratch, c->pade, (hipStream_t)hip_stream),
         "debug_expm");
  return LMAG_OK;
}

}  // extern "C"
