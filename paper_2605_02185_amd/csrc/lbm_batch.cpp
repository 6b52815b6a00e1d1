// Ensemble runtime of liblbm.so: many independent lattices advanced by one
// kernel launch per step (or per two to four steps with a multi-step
// variant) over the flattened tiles or wave tasks of every active case.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "lbm_internal.h"

namespace {

#define BTRY(call)                                                                            \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      char m_[256];                                                                           \
      snprintf(m_, sizeof m_, "%s: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
      return lbm::set_error(e_ == hipErrorOutOfMemory ? LBM_ERR_OOM : LBM_ERR_HIP, m_);       \
    }                                                                                         \
  } while (0)

}  // namespace

struct lbm_batch {
  int n = 0;
  hipStream_t stream = nullptr;
  std::vector<lbm_params> params;   // in budget order
  std::vector<int64_t> budget;      // in budget order, descending
  std::vector<int> slot_of_case;    // user index -> budget order
  std::vector<lbm::HostGeometry> hg;
  std::vector<lbm::CaseArgs> hcase;  // host mirror of d_cases
  lbm::CaseArgs* d_cases = nullptr;
  std::vector<void*> allocs;         // every device allocation
  int2* d_tiles = nullptr;
  std::vector<int> tile_prefix;      // tiles of the first k cases
  // multi-step variants: boundary and interior wave tasks of the first k
  // cases (prefix counts) in two device lists; the steps left over run the
  // one-step kernel of variant `single`
  int steps = 1;
  int single = 1;
  int2* d_gen_tasks = nullptr;
  int2* d_bulk_tasks = nullptr;
  size_t task_cap = 0;
  std::vector<int> gen_prefix, bulk_prefix;
  int partial_stride = 0;
  int variant = 1;
  int cur = 0;
  // buffer holding each case's state (budget order): cur while the case is
  // active, then the buffer of its last launch (a launch flips the buffers
  // once whatever its number of steps, so this is not the step parity)
  std::vector<int> case_cur;
  int64_t step = 0;                  // global step counter
  int pending = 0;                   // ring slots used since the last fold
  int pending_active = 0;            // active cases during the pending slots
  hipStream_t capture_stream = nullptr;
  // (cur, active) -> graph of kRing steps and whether it leaves the state in
  // the other buffer (an odd number of launches)
  std::map<std::pair<int, int>, std::pair<hipGraphExec_t, int>> graphs;
};

namespace {

lbm_status dmalloc(lbm_batch* b, void** p, size_t bytes) {
  BTRY(hipMalloc(p, bytes));
  b->allocs.push_back(*p);
  return LBM_OK;
}

int active_cases(const lbm_batch* b, int64_t step) {
  int k = 0;
  while (k < b->n && b->budget[k] > step) ++k;
  return k;
}

lbm_status fold(lbm_batch* b, hipStream_t s) {
  if (b->pending == 0) return LBM_OK;
  if (b->pending_active > 0)
    BTRY(lbm::launch_force_reduce_batch(b->d_cases, b->pending_active, b->pending, b->partial_stride, s));
  b->pending = 0;
  return LBM_OK;
}

// Steps of the next launch with `left` steps to go before the active set
// changes: the variant's steps when they fit into the force ring, else one.
int group(const lbm_batch* b, int64_t left) {
  return b->steps > 1 && left >= b->steps && b->pending + b->steps <= lbm::kRing ? b->steps : 1;
}

// k steps (1, or the variant's steps as group() allows) of the `active`
// leading cases on stream s; one launch either way.
lbm_status enqueue(lbm_batch* b, int active, hipStream_t s, int k = 1) {
  if (b->pending > 0 && active != b->pending_active) {
    lbm_status st = fold(b, s);
    if (st != LBM_OK) return st;
  }
  b->pending_active = active;
  if (active > 0) {
    if (k == 1)
      BTRY(lbm::launch_step_batch(b->d_cases, b->d_tiles, b->tile_prefix[active], b->cur, b->pending,
                                  b->partial_stride, b->single, s));
    else
      BTRY(lbm::launch_multistep_batch(b->d_cases, b->d_gen_tasks, b->gen_prefix[active], b->d_bulk_tasks,
                                       b->bulk_prefix[active], b->cur, b->pending, b->partial_stride,
                                       b->variant, s));
  }
  b->cur ^= 1;
  for (int c = 0; c < active; ++c) b->case_cur[c] = b->cur;
  b->step += k;
  b->pending += k;
  if (b->pending == lbm::kRing) return fold(b, s);
  return LBM_OK;
}

lbm_status set_variant(lbm_batch* b, int v) {
  b->variant = v;
  b->steps = lbm::multistep_batch_supported(v) ? lbm::variant(v).steps : 1;
  b->single = b->steps > 1 ? 1 : v;
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second.first);
  b->graphs.clear();
  std::vector<int2> tiles, gen, bulk;
  b->tile_prefix.assign(1, 0);
  b->gen_prefix.assign(1, 0);
  b->bulk_prefix.assign(1, 0);
  for (int i = 0; i < b->n; ++i) {
    lbm::CaseArgs& c = b->hcase[i];
    lbm::tiling_for_variant(c.g, b->single, &c.t);
    const int nt = c.t.ntx * c.t.nty;
    for (int t = 0; t < nt; ++t) tiles.push_back(make_int2(i, t));
    b->tile_prefix.push_back((int)tiles.size());
    if (b->steps > 1) {
      lbm::tiling_for_variant(c.g, v, &c.tm);
      const lbm::Variant& var = lbm::variant(v);
      const int per = (var.tile_y + var.sub - 1) / var.sub;
      const bool xper = b->params[i].x_periodic != 0;
      for (int seg = 0; seg < c.tm.nty; ++seg)
        for (int strip = 0; strip < c.tm.ntx; ++strip) {
          const int id = seg * c.tm.ntx + strip;
          if (lbm::interior_segment(c.g, c.tm, xper, strip, seg))
            bulk.push_back(make_int2(i, id));
          else
            for (int piece = 0; piece < per; ++piece) gen.push_back(make_int2(i, id * per + piece));
        }
    } else {
      c.tm = c.t;
    }
    b->gen_prefix.push_back((int)gen.size());
    b->bulk_prefix.push_back((int)bulk.size());
  }
  if (b->steps > 1 && std::max(gen.size(), bulk.size()) > b->task_cap) {
    // allocations stay until the ensemble is destroyed; grow only
    const size_t cap = std::max(gen.size(), bulk.size());
    lbm_status st = dmalloc(b, (void**)&b->d_gen_tasks, sizeof(int2) * std::max<size_t>(cap, 1));
    if (st != LBM_OK) return st;
    if ((st = dmalloc(b, (void**)&b->d_bulk_tasks, sizeof(int2) * std::max<size_t>(cap, 1))) != LBM_OK) return st;
    b->task_cap = cap;
  }
  BTRY(hipMemcpyAsync(b->d_cases, b->hcase.data(), sizeof(lbm::CaseArgs) * b->n, hipMemcpyHostToDevice,
                      b->stream));
  if (b->d_tiles) BTRY(hipMemcpyAsync(b->d_tiles, tiles.data(), sizeof(int2) * tiles.size(),
                                      hipMemcpyHostToDevice, b->stream));
  if (b->steps > 1) {
    if (!gen.empty())
      BTRY(hipMemcpyAsync(b->d_gen_tasks, gen.data(), sizeof(int2) * gen.size(), hipMemcpyHostToDevice, b->stream));
    if (!bulk.empty())
      BTRY(hipMemcpyAsync(b->d_bulk_tasks, bulk.data(), sizeof(int2) * bulk.size(), hipMemcpyHostToDevice,
                          b->stream));
  }
  BTRY(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

std::string tune_key(const lbm_batch* b) {
  std::string k = "batch";
  for (const auto& p : b->params) {
    char buf[96];
    snprintf(buf, sizeof buf, ":%dx%d/d%d/w%d/x%d/c%d", p.nx, p.ny, p.diameter, p.wall, p.x_periodic,
             p.collision);
    k += buf;
  }
  // keep keys short and stable: FNV-1a of the full description
  uint64_t h = 1469598103934665603ULL;
  for (unsigned char ch : k) h = (h ^ ch) * 1099511628211ULL;
  char out[64];
  snprintf(out, sizeof out, "batch-%d-%016llx", b->n, (unsigned long long)h);
  return out;
}

// The one-step ensemble launch walks its flattened tile list in order:
// variants with a remapped tile order are for single lattices only, and of
// the multi-step variants those with an ensemble kernel.
bool batch_capable(int v) {
  if (v < 1 || v > lbm::num_variants()) return false;
  const lbm::Variant& var = lbm::variant(v);
  return (var.steps == 1 && !var.remap_xcd) || lbm::multistep_batch_supported(v);
}

int cache_lookup(const char* path, const std::string& key) {
  if (!path) return 0;
  FILE* f = fopen(path, "r");
  if (!f) return 0;
  char k[256];
  int v = 0, found = 0;
  while (fscanf(f, "%255s %d", k, &v) == 2)
    if (key == k && batch_capable(v)) found = v;
  fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& key, int v) {
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d\n", key.c_str(), v);
  fclose(f);
}

void free_batch(lbm_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second.first);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  for (void* p : b->allocs) (void)hipFree(p);
  delete b;
}

// Starting variant before the autotuner runs (and if it cannot): four steps
// per launch with 8-row boundary pieces once the ensemble holds 2^22 nodes
// (on the 64 cylinder channels of 55 k - 882 k nodes, 26.3 M together, MRT:
// 152 k MLUPS against 83 k for one step per launch and 116-137 k for the
// other multi-step variants); smaller ensembles one step per launch.
int batch_default_variant(const lbm_batch* b) {
  int64_t nodes = 0;
  for (const auto& p : b->params) nodes += (int64_t)p.nx * p.ny;
  if (nodes < ((int64_t)1 << 22)) return 1;
  for (int v = 1; v <= lbm::num_variants(); ++v)
    if (std::strcmp(lbm::variant(v).name, "t4_h8_s8") == 0 && lbm::multistep_batch_supported(v)) return v;
  return 1;
}

lbm_status create_impl(const lbm_params* cases, const int64_t* budgets, int32_t n, void* stream,
                       lbm_batch** out) {
  lbm_batch* b = new lbm_batch();
  *out = b;
  b->n = n;
  b->stream = (hipStream_t)stream;
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  auto bud = [&](int i) { return budgets && budgets[i] >= 0 ? budgets[i] : INT64_MAX; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return bud(a) > bud(c); });
  b->slot_of_case.assign(n, 0);
  b->case_cur.assign(n, 0);
  for (int k = 0; k < n; ++k) {
    b->slot_of_case[order[k]] = k;
    b->params.push_back(cases[order[k]]);
    b->budget.push_back(bud(order[k]));
  }
  b->hg.resize(n);
  b->hcase.resize(n);
  int stride = 0;
  std::vector<int> link_off(n);
  for (int k = 0; k < n; ++k) {
    lbm_status st = lbm::build_geometry(&b->params[k], &b->hg[k]);
    if (st != LBM_OK) return st;
    link_off[k] = stride;
    stride += std::max(1, b->hg[k].g.n_link_nodes);
  }
  b->partial_stride = stride;
  double2* partials = nullptr;
  lbm_status st = dmalloc(b, (void**)&partials, sizeof(double2) * (size_t)stride * lbm::kRing);
  if (st != LBM_OK) return st;
  BTRY(hipMemsetAsync(partials, 0, sizeof(double2) * (size_t)stride * lbm::kRing, b->stream));
  size_t ntiles_max = 0;
  for (int k = 0; k < n; ++k) {
    const lbm_params& p = b->params[k];
    lbm::CaseArgs& c = b->hcase[k];
    c.g = b->hg[k].g;
    c.p = lbm::make_physics(&p);
    const size_t fbytes = (size_t)lbm::state_floats(c.g) * sizeof(float);
    for (int j = 0; j < 2; ++j) {
      if ((st = dmalloc(b, (void**)&c.buf[j], fbytes)) != LBM_OK) return st;
      BTRY(hipMemsetAsync(c.buf[j], 0, fbytes, b->stream));
    }
    if (!b->hg[k].flags.empty()) {
      uint16_t* fl = nullptr;
      int32_t* li = nullptr;
      if ((st = dmalloc(b, (void**)&fl, b->hg[k].flags.size() * sizeof(uint16_t))) != LBM_OK) return st;
      if ((st = dmalloc(b, (void**)&li, b->hg[k].link_index.size() * sizeof(int32_t))) != LBM_OK) return st;
      BTRY(hipMemcpyAsync(fl, b->hg[k].flags.data(), b->hg[k].flags.size() * sizeof(uint16_t),
                          hipMemcpyHostToDevice, b->stream));
      BTRY(hipMemcpyAsync(li, b->hg[k].link_index.data(), b->hg[k].link_index.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, b->stream));
      c.g.flags = fl;
      c.g.link_index = li;
      if (!b->hg[k].q.empty()) {
        float* q = nullptr;
        if ((st = dmalloc(b, (void**)&q, b->hg[k].q.size() * sizeof(float))) != LBM_OK) return st;
        BTRY(hipMemcpyAsync(q, b->hg[k].q.data(), b->hg[k].q.size() * sizeof(float), hipMemcpyHostToDevice,
                            b->stream));
        c.g.q = q;
      }
    }
    c.partial = partials + link_off[k];
    c.hist_cap = p.hist_capacity;
    if ((st = dmalloc(b, (void**)&c.hist, sizeof(double) * 2 * (size_t)c.hist_cap)) != LBM_OK) return st;
    BTRY(hipMemsetAsync(c.hist, 0, sizeof(double) * 2 * (size_t)c.hist_cap, b->stream));
    if ((st = dmalloc(b, (void**)&c.dev_step, sizeof(int64_t))) != LBM_OK) return st;
    if ((st = dmalloc(b, (void**)&c.bad_step, sizeof(int64_t))) != LBM_OK) return st;
    if ((st = dmalloc(b, (void**)&c.bad, sizeof(int))) != LBM_OK) return st;
    BTRY(hipMemsetAsync(c.dev_step, 0, sizeof(int64_t), b->stream));
    BTRY(hipMemsetAsync(c.bad_step, 0, sizeof(int64_t), b->stream));
    BTRY(lbm::launch_fill_int(c.bad, INT_MAX, b->stream));
    BTRY(lbm::launch_init_equilibrium(c.buf[0], c.g, p.u_in, p.perturb_amp, c.p.full_bb != 0, b->stream));
  }
  for (int v = 1; v <= lbm::num_variants(); ++v) {
    size_t total = 0;
    for (int k = 0; k < n; ++k) {
      lbm::Tiling t;
      lbm::tiling_for_variant(b->hcase[k].g, v, &t);
      total += (size_t)t.ntx * t.nty;
    }
    ntiles_max = std::max(ntiles_max, total);
  }
  if ((st = dmalloc(b, (void**)&b->d_cases, sizeof(lbm::CaseArgs) * n)) != LBM_OK) return st;
  if ((st = dmalloc(b, (void**)&b->d_tiles, sizeof(int2) * ntiles_max)) != LBM_OK) return st;
  return set_variant(b, batch_default_variant(b));
}

lbm_status check_case(const lbm_batch* b, int32_t c) {
  if (!b) return lbm::set_error(LBM_ERR_INVALID_ARG, "batch is NULL");
  if (c < 0 || c >= b->n) return lbm::set_error(LBM_ERR_INVALID_ARG, "case index out of range");
  return LBM_OK;
}

int64_t case_steps(const lbm_batch* b, int k) { return std::min(b->step, b->budget[k]); }

double time_variant(lbm_batch* b, int v, int steps) {
  if (set_variant(b, v) != LBM_OK) return 1e30;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return 1e30;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return 1e30;
  }
  const int active = b->n;
  for (int i = 0; i < 12;) {
    const int k = group(b, 12 - i);
    (void)enqueue(b, active, b->stream, k);
    i += k;
  }
  (void)hipEventRecord(e0, b->stream);
  for (int i = 0; i < steps;) {
    const int k = group(b, steps - i);
    (void)enqueue(b, active, b->stream, k);
    i += k;
  }
  (void)hipEventRecord(e1, b->stream);
  float ms = 1e30f;
  if (hipEventSynchronize(e1) == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
  (void)fold(b, b->stream);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

}  // namespace

extern "C" {

lbm_status lbm_batch_create(const lbm_params* cases, const int64_t* budgets, int32_t n, void* stream,
                            const char* tune_cache, lbm_batch** out) {
  if (!out || !cases || n < 1) return lbm::set_error(LBM_ERR_INVALID_ARG, "bad lbm_batch_create arguments");
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    lbm_status st = lbm_validate_params(&cases[i]);
    if (st != LBM_OK) return st;
  }
  lbm_batch* b = nullptr;
  lbm_status st = create_impl(cases, budgets, n, stream, &b);
  if (st == LBM_OK) {
    const hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) st = lbm::set_error(LBM_ERR_HIP, hipGetErrorString(e));
  }
  if (st == LBM_OK) {
    // autotune on a scratch ensemble of the same cases (this one is
    // untouched): every variant that can run an ensemble is timed over 48
    // steps (a multiple of 1, 2, 3 and 4 steps per launch) after 12 warm-up
    // steps, and the fastest is kept; a cache hit skips the timing
    const std::string key = tune_key(b);
    int best = cache_lookup(tune_cache, key);
    if (!best) {
      lbm_batch* scratch = nullptr;
      lbm_status s2 = create_impl(cases, nullptr, n, stream, &scratch);
      double tbest = 1e30;
      for (int v = 1; s2 == LBM_OK && v <= lbm::num_variants(); ++v) {
        if (!batch_capable(v)) continue;
        const double t = time_variant(scratch, v, 48);
        if (t < tbest) {
          tbest = t;
          best = v;
        }
      }
      free_batch(scratch);
      if (best) cache_store(tune_cache, key, best);
    }
    if (best) st = set_variant(b, best);
  }
  if (st != LBM_OK) {
    free_batch(b);
    return st;
  }
  *out = b;
  return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) { free_batch(b); }

int32_t lbm_batch_variant(const lbm_batch* b) { return b ? b->variant : 0; }

lbm_status lbm_batch_set_variant(lbm_batch* b, int32_t variant) {
  if (!b) return lbm::set_error(LBM_ERR_INVALID_ARG, "batch is NULL");
  if (!batch_capable(variant)) {
    char m[64];
    snprintf(m, sizeof m, "variant %d cannot run an ensemble", (int)variant);
    return lbm::set_error(LBM_ERR_INVALID_ARG, m);
  }
  lbm_status st = fold(b, b->stream);
  if (st != LBM_OK) return st;
  return set_variant(b, variant);
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t n) {
  if (!b || n < 0) return lbm::set_error(LBM_ERR_INVALID_ARG, "bad lbm_batch_step arguments");
  int64_t i = 0;
  while (i < n) {
    const int active = active_cases(b, b->step);
    if (active == 0) break;
    // steps until the active set changes
    const int64_t seg = std::min(n - i, b->budget[active - 1] - b->step);
    int64_t j = 0;
    while (j < seg && b->pending != 0) {
      const int k = group(b, seg - j);
      lbm_status st = enqueue(b, active, b->stream, k);
      if (st != LBM_OK) return st;
      j += k;
    }
    while (seg - j >= lbm::kRing) {
      const auto key = std::make_pair(b->cur, active);
      auto it = b->graphs.find(key);
      if (it == b->graphs.end()) {
        if (!b->capture_stream) BTRY(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
        const int cur0 = b->cur;
        const int64_t step0 = b->step;
        BTRY(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
        lbm_status st = LBM_OK;
        int launches = 0;
        for (int k = 0; k < lbm::kRing && st == LBM_OK; ++launches) {
          const int g = group(b, lbm::kRing - k);
          st = enqueue(b, active, b->capture_stream, g);
          k += g;
        }
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->capture_stream, &g);
        b->cur = cur0;
        for (int c = 0; c < active; ++c) b->case_cur[c] = cur0;
        b->step = step0;
        b->pending = 0;
        if (st != LBM_OK) {
          if (g) (void)hipGraphDestroy(g);
          return st;
        }
        if (e != hipSuccess) return lbm::set_error(LBM_ERR_HIP, hipGetErrorString(e));
        hipGraphExec_t ex = nullptr;
        const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e2 != hipSuccess) return lbm::set_error(LBM_ERR_HIP, hipGetErrorString(e2));
        it = b->graphs.emplace(key, std::make_pair(ex, launches & 1)).first;
      }
      BTRY(hipGraphLaunch(it->second.first, b->stream));
      b->cur ^= it->second.second;
      for (int c = 0; c < active; ++c) b->case_cur[c] = b->cur;
      b->step += lbm::kRing;
      j += lbm::kRing;
    }
    while (j < seg) {
      const int k = group(b, seg - j);
      lbm_status st = enqueue(b, active, b->stream, k);
      if (st != LBM_OK) return st;
      j += k;
    }
    i += seg;
  }
  return fold(b, b->stream);
}

lbm_status lbm_batch_sync(lbm_batch* b) {
  if (!b) return lbm::set_error(LBM_ERR_INVALID_ARG, "batch is NULL");
  BTRY(hipStreamSynchronize(b->stream));
  int bad = 0;
  for (int k = 0; k < b->n; ++k) {
    int64_t s = 0;
    BTRY(hipMemcpy(&s, b->hcase[k].bad_step, sizeof s, hipMemcpyDeviceToHost));
    bad += s != 0;
  }
  if (bad) {
    char m[96];
    snprintf(m, sizeof m, "%d case(s) diverged", bad);
    return lbm::set_error(LBM_ERR_DIVERGED, m);
  }
  return LBM_OK;
}

lbm_status lbm_batch_case_info(lbm_batch* b, int32_t c, int64_t* steps, int64_t* diverged_step) {
  lbm_status st = check_case(b, c);
  if (st != LBM_OK) return st;
  const int k = b->slot_of_case[c];
  BTRY(hipStreamSynchronize(b->stream));
  if (steps) *steps = case_steps(b, k);
  if (diverged_step) BTRY(hipMemcpy(diverged_step, b->hcase[k].bad_step, sizeof(int64_t), hipMemcpyDeviceToHost));
  return LBM_OK;
}

lbm_status lbm_batch_forces(lbm_batch* b, int32_t c, int64_t first, int64_t count, double* fx, double* fy,
                            double* cd, double* cl) {
  lbm_status st = check_case(b, c);
  if (st != LBM_OK) return st;
  const int k = b->slot_of_case[c];
  const lbm_params& p = b->params[k];
  const int64_t have = case_steps(b, k), cap = p.hist_capacity;
  if (count < 0 || first < 1) return lbm::set_error(LBM_ERR_INVALID_ARG, "first must be >= 1 and count >= 0");
  if (first + count - 1 > have || first <= have - cap)
    return lbm::set_error(LBM_ERR_RANGE, "requested force steps are not stored");
  if ((cd || cl) && !(p.u_in > 0 && p.diameter > 0))
    return lbm::set_error(LBM_ERR_INVALID_ARG, "coefficients need u_in > 0 and diameter > 0");
  BTRY(hipStreamSynchronize(b->stream));
  std::vector<double> h((size_t)2 * std::max<int64_t>(count, 1));
  int64_t done = 0;
  while (done < count) {
    const int64_t s = (first - 1 + done) % cap;
    const int64_t m = std::min(count - done, cap - s);
    BTRY(hipMemcpy(h.data() + 2 * done, b->hcase[k].hist + 2 * s, sizeof(double) * 2 * m,
                   hipMemcpyDeviceToHost));
    done += m;
  }
  const double q = 0.5 * p.u_in * p.u_in * p.diameter;  // Eq. 15, rho_in = 1
  for (int64_t i = 0; i < count; ++i) {
    if (fx) fx[i] = h[2 * i];
    if (fy) fy[i] = h[2 * i + 1];
    if (cd) cd[i] = h[2 * i] / q;
    if (cl) cl[i] = h[2 * i + 1] / q;
  }
  return LBM_OK;
}

lbm_status lbm_batch_fields(lbm_batch* b, int32_t c, float* rho, float* ux, float* uy, int on_device) {
  lbm_status st = check_case(b, c);
  if (st != LBM_OK) return st;
  const int k = b->slot_of_case[c];
  const lbm::CaseArgs& ca = b->hcase[k];
  // a case that stopped at its budget holds its state in the buffer of its
  // last launch (every case starts in buf[0])
  const float* state = ca.buf[b->case_cur[k]];
  const size_t n = (size_t)ca.g.nx * ca.g.ny;
  if (on_device) {
    BTRY(lbm::launch_fields(state, ca.g, rho, ux, uy, b->stream));
    BTRY(hipStreamSynchronize(b->stream));
    return LBM_OK;
  }
  float* d = nullptr;
  BTRY(hipMalloc(&d, 3 * n * sizeof(float)));
  hipError_t e = lbm::launch_fields(state, ca.g, d, d + n, d + 2 * n, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e == hipSuccess && rho) e = hipMemcpy(rho, d, n * sizeof(float), hipMemcpyDeviceToHost);
  if (e == hipSuccess && ux) e = hipMemcpy(ux, d + n, n * sizeof(float), hipMemcpyDeviceToHost);
  if (e == hipSuccess && uy) e = hipMemcpy(uy, d + 2 * n, n * sizeof(float), hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return lbm::set_error(LBM_ERR_HIP, hipGetErrorString(e));
  return LBM_OK;
}

lbm_status lbm_batch_get_populations(lbm_batch* b, int32_t c, void* buf, int dtype, int on_device) {
  lbm_status st = check_case(b, c);
  if (st != LBM_OK) return st;
  if (!buf || (dtype != 0 && dtype != 1)) return lbm::set_error(LBM_ERR_INVALID_ARG, "bad buffer or dtype");
  const int k = b->slot_of_case[c];
  const lbm::CaseArgs& ca = b->hcase[k];
  const float* own = ca.buf[b->case_cur[k]];
  const size_t bytes = (size_t)9 * ca.g.nx * ca.g.ny * (dtype ? 8 : 4);
  if (on_device) {
    BTRY(lbm::launch_pack(own, ca.g, buf, dtype, b->stream));
    BTRY(hipStreamSynchronize(b->stream));
    return LBM_OK;
  }
  void* d = nullptr;
  BTRY(hipMalloc(&d, bytes));
  hipError_t e = lbm::launch_pack(own, ca.g, d, dtype, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e == hipSuccess) e = hipMemcpy(buf, d, bytes, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return lbm::set_error(LBM_ERR_HIP, hipGetErrorString(e));
  return LBM_OK;
}

lbm_status lbm_batch_set_populations(lbm_batch* b, int32_t c, const void* buf, int dtype, int on_device) {
  lbm_status st = check_case(b, c);
  if (st != LBM_OK) return st;
  if (!buf || (dtype != 0 && dtype != 1)) return lbm::set_error(LBM_ERR_INVALID_ARG, "bad buffer or dtype");
  const int k = b->slot_of_case[c];
  const lbm::CaseArgs& ca = b->hcase[k];
  // the buffer the case's next step streams from (or its final state)
  float* own = ca.buf[b->case_cur[k]];
  const size_t bytes = (size_t)9 * ca.g.nx * ca.g.ny * (dtype ? 8 : 4);
  if (on_device) {
    BTRY(lbm::launch_unpack(buf, dtype, ca.g, own, b->stream));
    BTRY(hipStreamSynchronize(b->stream));
    return LBM_OK;
  }
  void* d = nullptr;
  BTRY(hipMalloc(&d, bytes));
  hipError_t e = hipMemcpyAsync(d, buf, bytes, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = lbm::launch_unpack(d, dtype, ca.g, own, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  (void)hipFree(d);
  if (e != hipSuccess) return lbm::set_error(LBM_ERR_HIP, hipGetErrorString(e));
  return LBM_OK;
}

}  // extern "C"
