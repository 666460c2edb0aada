// Batched estimation: many requests (different resident scenes, image sizes,
// N, d, spp) in one persistent render launch over (request, perturbation, run
// of tiles) work items, the whole sequence captured once in a HIP graph and
// replayed per batch.  Results are bit-identical to prdpt_grad_estimate of each
// request alone (same device functions, same summation order).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "ctx_internal.h"

namespace prdpt {

void batch_release(BatchState& b) {
  if (b.exec) hipGraphExecDestroy(b.exec);
  void* dev[] = {b.d_reqs,    b.d_meta,   b.d_tau,   b.d_c,   b.d_X,
                 b.d_partial, b.d_losses, b.d_grads, b.d_loss};
  for (void* p : dev)
    if (p) hipFree(p);
  void* host[] = {b.h_reqs, b.h_meta, b.h_grads, b.h_loss, b.h_losses};
  for (void* p : host)
    if (p) hipHostFree(p);
  if (b.ready) hipEventDestroy(b.ready);
  if (b.stream) hipStreamDestroy(b.stream);
  b = BatchState{};
}

namespace {

template <class T>
int grow_dev(T*& p, size_t& cap_field_unused, size_t n) {
  (void)cap_field_unused;
  if (p) {
    HIP_TRY(hipFree(p));
    p = nullptr;
  }
  if (dev_malloc((void**)&p, std::max<size_t>(1, n) * sizeof(T)) != hipSuccess) {
    p = nullptr;
    return fail(PRDPT_E_NOMEM, "device allocation for the batch failed");
  }
  return PRDPT_OK;
}

template <class T>
int grow_host(T*& p, size_t n) {
  if (p) {
    HIP_TRY(hipHostFree(p));
    p = nullptr;
  }
  if (pinned_malloc((void**)&p, std::max<size_t>(1, n) * sizeof(T)) != hipSuccess) {
    p = nullptr;
    return fail(PRDPT_E_NOMEM, "pinned host allocation for the batch failed");
  }
  return PRDPT_OK;
}

}  // namespace

// Create the batch stream on first use and grow device/pinned buffers to the
// given capacities (a capacity change invalidates the captured graph).
int ensure_batch(prdpt_ctx* ctx, BatchState& b, size_t n_req, size_t pairs, size_t rows,
                 size_t partial) {
  if (!b.stream) {
    HIP_TRY(hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&b.ready, hipEventDisableTiming));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, ctx->device));
    b.n_cu = prop.multiProcessorCount;
    size_t dummy = 0;
    int rc;
    if ((rc = grow_dev(b.d_meta, dummy, 1))) return rc;
    if ((rc = grow_host(b.h_meta, 1))) return rc;
  }
  bool changed = false;
  size_t dummy = 0;
  int rc;
  auto want = [](size_t need, size_t have) { return need > have ? std::max(need, have + have / 2) : 0; };
  if (size_t w = want(n_req, b.cap_req)) {
    HIP_TRY(hipStreamSynchronize(b.stream));
    if ((rc = grow_dev(b.d_reqs, dummy, w)) || (rc = grow_dev(b.d_grads, dummy, w * PRDPT_BATCH_MAX_PARAMS)) ||
        (rc = grow_dev(b.d_loss, dummy, w)) || (rc = grow_host(b.h_reqs, w)) ||
        (rc = grow_host(b.h_grads, w * PRDPT_BATCH_MAX_PARAMS)) || (rc = grow_host(b.h_loss, w)))
      return rc;
    b.cap_req = w;
    changed = true;
  }
  if (size_t w = want(pairs, b.cap_pairs)) {
    HIP_TRY(hipStreamSynchronize(b.stream));
    if ((rc = grow_dev(b.d_tau, dummy, w * PRDPT_BATCH_MAX_PARAMS)) ||
        (rc = grow_dev(b.d_c, dummy, w * PRDPT_BATCH_MAX_PARAMS)))
      return rc;
    b.cap_pairs = w;
    changed = true;
  }
  if (size_t w = want(rows, b.cap_rows)) {
    HIP_TRY(hipStreamSynchronize(b.stream));
    if ((rc = grow_dev(b.d_X, dummy, w * PRDPT_BATCH_MAX_PARAMS)) || (rc = grow_dev(b.d_losses, dummy, w)) ||
        (rc = grow_host(b.h_losses, w)))
      return rc;
    b.cap_rows = w;
    changed = true;
  }
  if (size_t w = want(partial, b.cap_partial)) {
    HIP_TRY(hipStreamSynchronize(b.stream));
    if ((rc = grow_dev(b.d_partial, dummy, w))) return rc;
    b.cap_partial = w;
    changed = true;
  }
  if (changed && b.exec) {
    HIP_TRY(hipGraphExecDestroy(b.exec));
    b.exec = nullptr;
  }
  return PRDPT_OK;
}

namespace {

int check_one(prdpt_ctx* ctx, const prdpt_request& r) {
  const prdpt_scene* s = r.scene;
  if (!s || s->ctx != ctx) return PRDPT_E_ARG;
  if (!r.ref || !r.theta || !r.sigma || !r.grad_out) return PRDPT_E_ARG;
  if (r.N < 2 || (r.N & 1) || r.N > (1 << 20)) return PRDPT_E_ARG;
  if (r.est < PRDPT_EST_GAUSS || r.est > PRDPT_EST_IS_PERDIM) return PRDPT_E_ARG;
  if (s->hdr.n_param > PRDPT_BATCH_MAX_PARAMS) return PRDPT_E_ARG;
  for (int j = 0; j < s->hdr.n_param; ++j) {
    if (!std::isfinite(r.theta[j])) return PRDPT_E_ARG;
    if (!(r.sigma[j] > 0.0f) || !std::isfinite(r.sigma[j])) return PRDPT_E_ARG;
  }
  return PRDPT_OK;
}

int launch_sequence(BatchState& b, int render_blocks, int rot, int max_sph) {
  HIP_TRY(launch_batch(b.stream, b.d_reqs, b.d_meta, render_blocks, rot, max_sph, b.d_tau,
                       b.d_c, b.d_X, b.d_partial, b.d_losses, b.d_grads, b.d_loss));
  return PRDPT_OK;
}

}  // namespace

// Enqueue the valid requests of `reqs` as one batch on b's stream (tables,
// graph replay or direct launches, asynchronous copies of the results into
// pinned memory).  Per-request status in reqs[i].status; `ok` receives the
// indices of the requests that run, in table order.  If `t0`/`t1` are given,
// events bracket the device work.
int batch_enqueue(prdpt_ctx* ctx, BatchState& b, prdpt_request* reqs, int n, std::vector<int>& ok,
                  hipEvent_t t0, hipEvent_t t1) {
  ok.clear();
  for (int i = 0; i < n; ++i) {
    reqs[i].status = check_one(ctx, reqs[i]);
    if (reqs[i].status == PRDPT_OK) ok.push_back(i);
  }
  if (ok.empty()) return PRDPT_OK;
  // largest work per item first: shortens the tail of the persistent launch
  std::stable_sort(ok.begin(), ok.end(), [&](int a, int c) {
    const SceneHdr& ha = reqs[a].scene->hdr;
    const SceneHdr& hc = reqs[c].scene->hdr;
    return (long long)ha.spp * (ha.B + 1) > (long long)hc.spp * (hc.B + 1);
  });
  size_t pairs = 0, rows = 0, partial = 0, items = 0;
  const int tpi = b.tiles_per_item;
  for (int i : ok) {
    const SceneHdr& h = reqs[i].scene->hdr;
    const int nt = render_tiles(h.W, h.H, h.tile_log2);
    pairs += reqs[i].N / 2;
    rows += reqs[i].N;
    partial += (size_t)reqs[i].N * nt;
    items += (size_t)reqs[i].N * ((nt + tpi - 1) / tpi);
  }
  if (items >= (1u << 31) || partial >= (1u << 31)) return fail(PRDPT_E_ARG, "batch too large");
  if (int rc = ensure_batch(ctx, b, ok.size(), pairs, rows, partial)) return rc;
  // request table
  int item_base = 0, pair_base = 0, row_base = 0, partial_base = 0;
  for (size_t q = 0; q < ok.size(); ++q) {
    const prdpt_request& r = reqs[ok[q]];
    const SceneHdr& h = r.scene->hdr;
    BatchReq& t = b.h_reqs[q];
    std::memset(&t, 0, sizeof(t));
    t.scene = r.scene->dev();
    t.ref = r.ref;
    t.W = h.W;
    t.H = h.H;
    t.N = r.N;
    t.d = h.n_param;
    t.n_tiles = render_tiles(h.W, h.H, h.tile_log2);
    t.items_per_row = (t.n_tiles + tpi - 1) / tpi;
    t.est = r.est;
    t.k0 = (uint32_t)r.seed;
    t.k1 = (uint32_t)(r.seed >> 32);
    t.item_base = item_base;
    t.pair_base = pair_base;
    t.row_base = row_base;
    t.partial_base = partial_base;
    t.cd = chi_mean(t.d);
    t.sqrt2pi = std::sqrt(2.0 * M_PI);
    t.inv_den = 1.0 / (3.0 * (double)h.W * (double)h.H);
    for (int j = 0; j < t.d; ++j) {
      t.theta[j] = r.theta[j];
      t.sigma[j] = r.sigma[j];
    }
    item_base += r.N * t.items_per_row;
    pair_base += r.N / 2;
    row_base += r.N;
    partial_base += r.N * t.n_tiles;
  }
  BatchMeta& m = *b.h_meta;
  std::memset(&m, 0, sizeof(m));
  m.n_req = (int)ok.size();
  m.total_pairs = pair_base;
  m.total_items = item_base;
  m.total_rows = row_base;
  m.tiles_per_item = tpi;
  int rot = 0;  // the render variant that applies instance rotations
  int max_sph = 0;
  for (int i : ok) {
    rot |= reqs[i].scene->hdr.has_rot;
    max_sph = std::max(max_sph, reqs[i].scene->hdr.n_sph);
  }
  // blocks_per_cu 0: every work-group the CUs hold at once
  const int render_blocks = b.blocks_per_cu > 0 ? std::max(1, b.n_cu * b.blocks_per_cu)
                                                : std::max(1, batch_grid_limit(rot, max_sph));
  // order after earlier work on the context stream (e.g. reference uploads)
  HIP_TRY(hipEventRecord(b.ready, ctx->stream));
  HIP_TRY(hipStreamWaitEvent(b.stream, b.ready, 0));
  HIP_TRY(hipMemcpyAsync(b.d_reqs, b.h_reqs, sizeof(BatchReq) * ok.size(), hipMemcpyHostToDevice, b.stream));
  HIP_TRY(hipMemcpyAsync(b.d_meta, b.h_meta, sizeof(BatchMeta), hipMemcpyHostToDevice, b.stream));
  if (t0) HIP_TRY(hipEventRecord(t0, b.stream));
  if (b.use_graph) {
    if (b.exec && (b.graph_blocks != render_blocks || b.graph_rot != rot || b.graph_sph != max_sph)) {
      HIP_TRY(hipGraphExecDestroy(b.exec));
      b.exec = nullptr;
    }
    if (!b.exec) {
      hipGraph_t g = nullptr;
      HIP_TRY(hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal));
      const int rc = launch_sequence(b, render_blocks, rot, max_sph);
      hipError_t e = hipStreamEndCapture(b.stream, &g);
      if (rc) return rc;
      if (e != hipSuccess) return fail(PRDPT_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&b.exec, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (e != hipSuccess) {
        b.exec = nullptr;
        return fail(PRDPT_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
      }
      b.graph_blocks = render_blocks;
      b.graph_rot = rot;
      b.graph_sph = max_sph;
    }
    HIP_TRY(hipGraphLaunch(b.exec, b.stream));
  } else {
    if (int rc = launch_sequence(b, render_blocks, rot, max_sph)) return rc;
  }
  if (t1) HIP_TRY(hipEventRecord(t1, b.stream));
  HIP_TRY(hipMemcpyAsync(b.h_grads, b.d_grads, sizeof(double) * PRDPT_BATCH_MAX_PARAMS * ok.size(),
                         hipMemcpyDeviceToHost, b.stream));
  HIP_TRY(hipMemcpyAsync(b.h_loss, b.d_loss, sizeof(double) * ok.size(), hipMemcpyDeviceToHost, b.stream));
  HIP_TRY(hipMemcpyAsync(b.h_losses, b.d_losses, sizeof(double) * rows, hipMemcpyDeviceToHost, b.stream));
  return PRDPT_OK;
}

// Scatter the results of a finished batch (b's stream complete) to the requests.
void batch_collect(BatchState& b, prdpt_request* reqs, const std::vector<int>& ok) {
  for (size_t q = 0; q < ok.size(); ++q) {
    prdpt_request& r = reqs[ok[q]];
    const BatchReq& t = b.h_reqs[q];
    std::memcpy(r.grad_out, b.h_grads + q * PRDPT_BATCH_MAX_PARAMS, sizeof(double) * t.d);
    if (r.loss_out) *r.loss_out = b.h_loss[q];
    if (r.losses_out) std::memcpy(r.losses_out, b.h_losses + t.row_base, sizeof(double) * r.N);
  }
}

namespace {

// Runs the valid requests of `reqs` on the context's batch state, synchronously.
int run_batch(prdpt_ctx* ctx, prdpt_request* reqs, int n, double* device_ms) {
  BatchState& b = ctx->batch;
  if (int rc = ensure_batch(ctx, b, 1, 1, 1, 1)) return rc;
  std::vector<int> ok;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (device_ms) {
    HIP_TRY(hipEventCreate(&t0));
    HIP_TRY(hipEventCreate(&t1));
  }
  int rc = batch_enqueue(ctx, b, reqs, n, ok, t0, t1);
  if (rc == PRDPT_OK && !ok.empty()) {
    hipError_t e = hipStreamSynchronize(b.stream);
    if (e != hipSuccess) rc = fail(PRDPT_E_HIP, std::string("batch: ") + hipGetErrorString(e));
  }
  if (rc == PRDPT_OK && device_ms) {
    float ms = 0.0f;
    if (!ok.empty() && hipEventElapsedTime(&ms, t0, t1) == hipSuccess) *device_ms = ms;
  }
  if (t0) hipEventDestroy(t0);
  if (t1) hipEventDestroy(t1);
  if (rc == PRDPT_OK) batch_collect(b, reqs, ok);
  return rc;
}

// size class of a batch for the autotuner cache: CU count, log2 of the camera
// paths, log2 of the request count
std::string size_key(prdpt_ctx* ctx, const prdpt_request* reqs, int n) {
  double paths = 0.0;
  int valid = 0;
  for (int i = 0; i < n; ++i) {
    if (!reqs[i].scene) continue;
    const SceneHdr& h = reqs[i].scene->hdr;
    paths += (double)reqs[i].N * h.W * h.H * h.spp;
    ++valid;
  }
  std::ostringstream os;
  os << "cu" << ctx->batch.n_cu << "_paths2e" << (int)std::floor(std::log2(std::max(1.0, paths)))
     << "_req2e" << (int)std::floor(std::log2(std::max(1, valid)));
  return os.str();
}

bool read_cache(const char* path, const std::string& key, int* bpc, int* tpi, double* ms) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  const std::string tag = "\"key\": \"" + key + "\"";
  while (std::getline(f, line)) {
    if (line.find(tag) == std::string::npos) continue;
    int a = 0, b = 0;
    double t = 0.0;
    const char* p = std::strstr(line.c_str(), "\"blocks_per_cu\":");
    const char* q = std::strstr(line.c_str(), "\"tiles_per_item\":");
    const char* r = std::strstr(line.c_str(), "\"ms\":");
    if (!p || !q || !r) continue;
    if (std::sscanf(p, "\"blocks_per_cu\": %d", &a) != 1 || std::sscanf(q, "\"tiles_per_item\": %d", &b) != 1 ||
        std::sscanf(r, "\"ms\": %lf", &t) != 1)
      continue;
    *bpc = a;
    *tpi = b;
    *ms = t;
    return true;
  }
  return false;
}

void write_cache(const char* path, const std::string& key, int bpc, int tpi, double ms) {
  if (!path) return;
  std::vector<std::string> keep;
  {
    std::ifstream f(path);
    std::string line;
    const std::string tag = "\"key\": \"" + key + "\"";
    while (std::getline(f, line))
      if (!line.empty() && line.find(tag) == std::string::npos) keep.push_back(line);
  }
  std::ostringstream os;
  os.precision(17);  // the stored time reads back exactly
  os << "{\"key\": \"" << key << "\", \"blocks_per_cu\": " << bpc << ", \"tiles_per_item\": " << tpi
     << ", \"ms\": " << ms << "}";
  keep.push_back(os.str());
  std::ofstream f(path, std::ios::trunc);
  for (auto& l : keep) f << l << "\n";
}

}  // namespace
}  // namespace prdpt

using namespace prdpt;

extern "C" {

int prdpt_batch_estimate(prdpt_ctx* ctx, prdpt_request* reqs, int n) {
  if (!ctx || (!reqs && n > 0) || n < 0) return fail(PRDPT_E_ARG, "null argument");
  if (n == 0) return PRDPT_OK;
  std::lock_guard<std::mutex> g(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->device));
  return run_batch(ctx, reqs, n, nullptr);
}

int prdpt_batch_config(prdpt_ctx* ctx, int blocks_per_cu, int tiles_per_item, int use_graph) {
  if (!ctx) return fail(PRDPT_E_ARG, "ctx is null");
  if (blocks_per_cu < 0 || blocks_per_cu > 64 || tiles_per_item < 1 || tiles_per_item > 4096)
    return fail(PRDPT_E_ARG, "blocks_per_cu in 0..64, tiles_per_item in 1..4096");
  std::lock_guard<std::mutex> g(ctx->mu);
  BatchState& b = ctx->batch;
  if (b.exec && (b.blocks_per_cu != blocks_per_cu || b.tiles_per_item != tiles_per_item)) {
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipStreamSynchronize(b.stream));
    HIP_TRY(hipGraphExecDestroy(b.exec));
    b.exec = nullptr;
  }
  b.blocks_per_cu = blocks_per_cu;
  b.tiles_per_item = tiles_per_item;
  b.use_graph = use_graph ? 1 : 0;
  return PRDPT_OK;
}

int prdpt_batch_autotune(prdpt_ctx* ctx, prdpt_request* reqs, int n, const char* cache_path,
                         int* best_blocks_per_cu, int* best_tiles_per_item, double* best_ms) {
  if (!ctx || !reqs || n < 1) return fail(PRDPT_E_ARG, "null argument");
  std::lock_guard<std::mutex> g(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->device));
  BatchState& b = ctx->batch;
  if (int rc = ensure_batch(ctx, b, 1, 1, 1, 1)) return rc;
  const std::string key = size_key(ctx, reqs, n);
  int bpc = 0, tpi = 0;
  double ms = 0.0;
  if (!read_cache(cache_path, key, &bpc, &tpi, &ms)) {
    const int cand_bpc[] = {4, 8, 12, 16, 20, 24};
    const int cand_tpi[] = {1, 2, 4};
    double best = 1e300;
    for (int cb : cand_bpc)
      for (int ct : cand_tpi) {
        b.blocks_per_cu = cb;
        b.tiles_per_item = ct;
        if (b.exec) {
          HIP_TRY(hipStreamSynchronize(b.stream));
          HIP_TRY(hipGraphExecDestroy(b.exec));
          b.exec = nullptr;
        }
        double t = 0.0;
        if (int rc = run_batch(ctx, reqs, n, &t)) return rc;  // warm-up and capture
        double tsum = 0.0;
        for (int rep = 0; rep < 2; ++rep) {
          if (int rc = run_batch(ctx, reqs, n, &t)) return rc;
          tsum += t;
        }
        if (tsum / 2 < best) {
          best = tsum / 2;
          bpc = cb;
          tpi = ct;
        }
      }
    ms = best;
    write_cache(cache_path, key, bpc, tpi, ms);
  }
  if (b.exec && (b.blocks_per_cu != bpc || b.tiles_per_item != tpi)) {
    HIP_TRY(hipStreamSynchronize(b.stream));
    HIP_TRY(hipGraphExecDestroy(b.exec));
    b.exec = nullptr;
  }
  b.blocks_per_cu = bpc;
  b.tiles_per_item = tpi;
  if (best_blocks_per_cu) *best_blocks_per_cu = bpc;
  if (best_tiles_per_item) *best_tiles_per_item = tpi;
  if (best_ms) *best_ms = ms;
  return PRDPT_OK;
}

}  // extern "C"
