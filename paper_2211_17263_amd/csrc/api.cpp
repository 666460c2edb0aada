// C ABI of the estimator: contexts, resident scenes and the estimator calls.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ctx_internal.h"

using namespace prdpt;

namespace {
thread_local std::string g_err;
}  // namespace

int prdpt::fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

namespace {
// allocation-failure injection: < 0 off; otherwise the number of allocations
// still allowed to succeed before every later one fails
std::atomic<int64_t> g_alloc_budget{-1};

bool alloc_allowed() {
  int64_t left = g_alloc_budget.load();
  while (left >= 0) {
    if (left == 0) return false;
    if (g_alloc_budget.compare_exchange_weak(left, left - 1)) return true;
  }
  return true;
}
}  // namespace

hipError_t prdpt::dev_malloc(void** p, size_t bytes) {
  *p = nullptr;
  if (!alloc_allowed()) return hipErrorOutOfMemory;
  return hipMalloc(p, bytes);
}

hipError_t prdpt::pinned_malloc(void** p, size_t bytes) {
  *p = nullptr;
  if (!alloc_allowed()) return hipErrorOutOfMemory;
  return hipHostMalloc(p, bytes, hipHostMallocDefault);
}

namespace {

template <class T>
int ensure(prdpt_ctx* ctx, DevBuf<T>& b, size_t n) {
  if (n == 0) n = 1;
  if (b.n >= n) return PRDPT_OK;
  if (b.p) {
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipFree(b.p));
    b.p = nullptr;
    b.n = 0;
  }
  size_t want = n + n / 2;
  if (dev_malloc((void**)&b.p, want * sizeof(T)) != hipSuccess) {
    b.p = nullptr;
    return fail(PRDPT_E_NOMEM, "device allocation of scratch failed");
  }
  b.n = want;
  return PRDPT_OK;
}

hipEvent_t take_event(prdpt_ctx* ctx) {
  if (!ctx->pool.empty()) {
    hipEvent_t e = ctx->pool.back();
    ctx->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// launch the fused render kernel, bracketed by timing events when enabled
hipError_t timed_render(prdpt_ctx* ctx, const prdpt_scene* s, const float* X, int nk, int d, int tag,
                        uint64_t seed, const float* ref, float* img, float* partial, int crn,
                        int* work, bool allow_timing = true) {
  const DevScene sc = s->dev();
  const int W = s->hdr.W, H = s->hdr.H;
  hipEvent_t a = nullptr, b = nullptr;
  if (ctx->timing && allow_timing) {
    a = take_event(ctx);
    b = take_event(ctx);
    if (a && b) {
      hipError_t e = hipEventRecord(a, ctx->stream);
      if (e != hipSuccess) return e;
    }
  }
  hipError_t e = launch_render(ctx->stream, sc, W, H, s->hdr.tile_log2, X, nk, d, tag, seed, ref, img,
                               partial, nullptr,
                               work, s->d_tile_order, s->d_tile_cost, crn, s->hdr.has_rot,
                               s->hdr.n_sph);
  if (e != hipSuccess) return e;
  if (a && b) {
    e = hipEventRecord(b, ctx->stream);
    if (e != hipSuccess) return e;
    ctx->pending.emplace_back(a, b);
  }
  // the next render of this scene takes its costliest tiles first; when every
  // work item of a launch like this one is resident at once, the order cannot
  // matter and the sort (a launch of its own) is skipped
  if ((long long)nk * s->n_tiles <=
      (long long)render_grid_limit(s->hdr.has_rot, s->hdr.n_sph, s->hdr.tile_log2))
    return hipSuccess;
  return launch_tile_order(ctx->stream, s->d_tile_cost, s->d_tile_order, s->n_tiles);
}

int check_request(const prdpt_scene* s, const float* theta, const float* sigma, int N,
                  bool host_vectors) {
  if (!s) return fail(PRDPT_E_ARG, "scene is null");
  if (!theta || !sigma) return fail(PRDPT_E_ARG, "theta/sigma is null");
  if (N < 2 || (N & 1)) return fail(PRDPT_E_ARG, "N must be even and >= 2");
  if (N > (1 << 20)) return fail(PRDPT_E_ARG, "N too large");
  // (perturbation, tile) work items are counted in 32 bits
  if ((long long)N * render_tiles(s->hdr.W, s->hdr.H, s->hdr.tile_log2) >= (1ll << 31))
    return fail(PRDPT_E_ARG, "N x pixel tiles must stay below 2^31");
  if (host_vectors) {
    for (int j = 0; j < s->hdr.n_param; ++j) {
      if (!std::isfinite(theta[j])) return fail(PRDPT_E_ARG, "theta must be finite");
      if (!(sigma[j] > 0.0f) || !std::isfinite(sigma[j]))
        return fail(PRDPT_E_ARG, "sigma must be positive and finite");
    }
  }
  return PRDPT_OK;
}

int check_est(int est) {
  const int mode = est & ~(PRDPT_EST_INDEPENDENT | PRDPT_EST_STRATIFIED);
  if (mode != PRDPT_EST_GAUSS && mode != PRDPT_EST_IS && mode != PRDPT_EST_IS_PERDIM)
    return fail(PRDPT_E_ARG, "unknown estimator mode");
  if ((est & PRDPT_EST_STRATIFIED) && !(est & PRDPT_EST_INDEPENDENT))
    return fail(PRDPT_E_ARG, "stratified draws need PRDPT_EST_INDEPENDENT");
  return PRDPT_OK;
}

// perturbation draws of an estimate with N renders: pairs, or N independent draws
int n_draws(int est, int N) { return (est & PRDPT_EST_INDEPENDENT) ? N : N / 2; }

// Scratch for one request with N renders; returns status.
int prepare(prdpt_ctx* ctx, int N, int d, int n_tiles) {
  int P = N / 2, rc;
  if ((rc = ensure(ctx, ctx->X, (size_t)N * d))) return rc;
  (void)P;  // tau and c hold up to N rows (independent draws)
  if ((rc = ensure(ctx, ctx->tau, (size_t)N * d))) return rc;
  if ((rc = ensure(ctx, ctx->c, (size_t)N * d))) return rc;
  if ((rc = ensure(ctx, ctx->partial, (size_t)N * n_tiles))) return rc;
  if ((rc = ensure(ctx, ctx->losses, (size_t)N))) return rc;
  if ((rc = ensure(ctx, ctx->grad, (size_t)d))) return rc;
  if ((rc = ensure(ctx, ctx->loss, 1))) return rc;
  if ((rc = ensure(ctx, ctx->theta, (size_t)d))) return rc;
  if ((rc = ensure(ctx, ctx->sigma, (size_t)d))) return rc;
  if ((rc = ensure(ctx, ctx->work, 1))) return rc;
  return PRDPT_OK;
}

// device arrays of one estimate: parameter rows, draws, weights, per-tile
// partial losses, per-image losses and the render's work counter
struct EstimateBufs {
  float* X;
  float* tau;
  double* c;
  float* partial;
  double* losses;
  int* work;
};

// enqueue tau + fused render/loss + losses + combine on the context stream
// into the given buffers (c_dev / losses_dev, when not null, replace b.c /
// b.losses); allow_timing = false records no timing events
int enqueue_into(prdpt_scene* s, const float* ref, const float* theta_dev, const float* sigma_dev,
                 int N, uint64_t seed, int est, double* grad_dev, double* loss_dev,
                 double* losses_dev, double* c_dev, const EstimateBufs& b, bool allow_timing) {
  prdpt_ctx* ctx = s->ctx;
  const SceneHdr& h = s->hdr;
  const int d = h.n_param;
  const int indep = (est & PRDPT_EST_INDEPENDENT) != 0;
  const int rows = n_draws(est, N);
  const int n_tiles = render_tiles(h.W, h.H, h.tile_log2);
  double* c = c_dev ? c_dev : b.c;
  double* L = losses_dev ? losses_dev : b.losses;
  HIP_TRY(launch_tau(ctx->stream, est, d, rows, seed, sigma_dev, theta_dev, chi_mean(d),
                     std::sqrt(2.0 * M_PI), b.tau, c, b.X));
  HIP_TRY(timed_render(ctx, s, b.X, N, d, kTagPath, seed, ref, nullptr, b.partial, indep ? 0 : 1,
                       b.work, allow_timing));
  HIP_TRY(launch_losses(ctx->stream, b.partial, n_tiles, N, h.W * h.H, L));
  HIP_TRY(launch_combine(ctx->stream, rows, d, indep, c, L, nullptr, grad_dev, loss_dev));
  return PRDPT_OK;
}

// the same on the context's own scratch (allocated or grown on demand)
int enqueue_estimate(prdpt_scene* s, const float* ref, const float* theta_dev,
                     const float* sigma_dev, int N, uint64_t seed, int est, double* grad_dev,
                     double* loss_dev, double* losses_dev, double* c_dev) {
  prdpt_ctx* ctx = s->ctx;
  const SceneHdr& h = s->hdr;
  if (int rc = prepare(ctx, N, h.n_param, render_tiles(h.W, h.H, h.tile_log2))) return rc;
  const EstimateBufs b{ctx->X.p, ctx->tau.p, ctx->c.p, ctx->partial.p, ctx->losses.p, ctx->work.p};
  return enqueue_into(s, ref, theta_dev, sigma_dev, N, seed, est, grad_dev, loss_dev, losses_dev,
                      c_dev, b, true);
}

// pinned host staging of at least n elements (hipHostMalloc; grows only)
template <class T>
int ensure_pinned(prdpt_ctx* ctx, T*& p, size_t& cap, size_t n) {
  if (cap >= n) return PRDPT_OK;
  if (p) {
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipHostFree(p));
    p = nullptr;
    cap = 0;
  }
  if (pinned_malloc((void**)&p, n * sizeof(T)) != hipSuccess) {
    p = nullptr;
    return fail(PRDPT_E_NOMEM, "pinned host allocation failed");
  }
  cap = n;
  return PRDPT_OK;
}

int upload_vectors(prdpt_ctx* ctx, const float* theta, const float* sigma, int d) {
  HIP_TRY(hipMemcpyAsync(ctx->theta.p, theta, sizeof(float) * d, hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(hipMemcpyAsync(ctx->sigma.p, sigma, sizeof(float) * d, hipMemcpyHostToDevice, ctx->stream));
  return PRDPT_OK;
}

}  // namespace

extern "C" {

const char* prdpt_last_error(void) { return g_err.c_str(); }

int prdpt_debug_fail_allocations(int64_t after) {
  g_alloc_budget.store(after < 0 ? -1 : after);
  return PRDPT_OK;
}

int prdpt_ctx_create(int device, void* stream, size_t hbm_budget, prdpt_ctx** out) {
  if (!out) return fail(PRDPT_E_ARG, "out is null");
  *out = nullptr;
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(PRDPT_E_ARG, "no such device");
  HIP_TRY(hipSetDevice(device));
  prdpt_ctx* ctx = new prdpt_ctx();
  ctx->device = device;
  ctx->budget = hbm_budget;
  ctx->stream = (hipStream_t)stream;  // NULL: the device's null stream
  // this device's copy of the allocation-free estimate's scratch array (a
  // failed lookup only disables that entry point)
  ctx->scratch_status = noalloc_scratch(device, &ctx->scratch);
  if (ctx->scratch_status != hipSuccess) ctx->scratch = nullptr;
  *out = ctx;
  return PRDPT_OK;
}

int prdpt_ctx_set_stream(prdpt_ctx* ctx, void* stream) {
  if (!ctx) return fail(PRDPT_E_ARG, "ctx is null");
  std::lock_guard<std::mutex> g(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  ctx->stream = (hipStream_t)stream;
  return PRDPT_OK;
}

int prdpt_ctx_destroy(prdpt_ctx* ctx) {
  if (!ctx) return fail(PRDPT_E_ARG, "ctx is null");
  if (ctx->n_scenes) return fail(PRDPT_E_ARG, "destroy the context's scenes first");
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  void* bufs[] = {ctx->X.p, ctx->tau.p, ctx->partial.p, ctx->theta.p, ctx->sigma.p,
                  ctx->images.p, ctx->dp_partial.p,
                  ctx->c.p, ctx->losses.p, ctx->grad.p, ctx->loss.p, ctx->counters.p, ctx->work.p,
                  ctx->vin.p, ctx->vout.p};
  for (void* b : bufs)
    if (b) hipFree(b);
  if (ctx->h_vin) hipHostFree(ctx->h_vin);
  if (ctx->h_vout) hipHostFree(ctx->h_vout);
  for (auto& pr : ctx->pending) {
    hipEventDestroy(pr.first);
    hipEventDestroy(pr.second);
  }
  for (hipEvent_t e : ctx->pool) hipEventDestroy(e);
  batch_release(ctx->batch);
  delete ctx;
  return PRDPT_OK;
}

int prdpt_ctx_resident_bytes(prdpt_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return fail(PRDPT_E_ARG, "null argument");
  std::lock_guard<std::mutex> g(ctx->mu);
  *bytes = ctx->resident;
  return PRDPT_OK;
}

int prdpt_ctx_synchronize(prdpt_ctx* ctx) {
  if (!ctx) return fail(PRDPT_E_ARG, "ctx is null");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return PRDPT_OK;
}

}  // extern "C"

// Validate a scene description, build its header and BVHs on the host.
int prdpt::build_host_scene(const prdpt_scene_desc* D, HostScene& hs) {
  if (!D) return fail(PRDPT_E_ARG, "null argument");
  // ---- validation ----
  if (D->width < 1 || D->height < 1 || D->width > PRDPT_MAX_SIDE || D->height > PRDPT_MAX_SIDE)
    return fail(PRDPT_E_SCENE, "image size out of range");
  if (D->spp < 1 || D->spp > 65536) return fail(PRDPT_E_SCENE, "spp out of range");
  if (D->max_bounces < 0 || D->max_bounces > PRDPT_MAX_BOUNCES)
    return fail(PRDPT_E_SCENE, "max_bounces out of range");
  if (D->n_params < 1 || D->n_params > PRDPT_MAX_PARAMS || !D->bindings)
    return fail(PRDPT_E_SCENE, "n_params out of range");
  if (D->n_materials < 1 || D->n_materials > PRDPT_MAX_MATERIALS || !D->mat_type || !D->mat_rgb ||
      !D->mat_ior)
    return fail(PRDPT_E_SCENE, "materials missing or too many");
  if (D->n_spheres < 0 || D->n_spheres > PRDPT_MAX_SPHERES || D->n_quads < 0 ||
      D->n_quads > PRDPT_MAX_QUADS || D->n_point_lights < 0 ||
      D->n_point_lights > PRDPT_MAX_POINT_LIGHTS || D->n_meshes < 0 || D->n_triangles < 0)
    return fail(PRDPT_E_SCENE, "primitive counts out of range");
  if ((D->n_spheres && (!D->spheres || !D->sphere_mat)) || (D->n_quads && (!D->quads || !D->quad_mat)) ||
      (D->n_point_lights && !D->point_lights) ||
      (D->n_meshes && (!D->mesh_offset || !D->mesh_mat || !D->mesh_translation)) ||
      (D->n_triangles && !D->triangles))
    return fail(PRDPT_E_SCENE, "null array for a non-empty primitive list");
  for (int i = 0; i < D->n_materials; ++i)
    if (D->mat_type[i] < 0 || D->mat_type[i] > 2) return fail(PRDPT_E_SCENE, "bad material type");
  auto mat_ok = [&](int m) { return m >= 0 && m < D->n_materials; };
  for (int i = 0; i < D->n_spheres; ++i) {
    if (!mat_ok(D->sphere_mat[i]) || D->mat_type[D->sphere_mat[i]] == PRDPT_MAT_EMISSIVE)
      return fail(PRDPT_E_SCENE, "sphere material must be diffuse or dielectric");
    if (!(D->spheres[4 * i + 3] > 0.0f)) return fail(PRDPT_E_SCENE, "sphere radius must be > 0");
  }
  for (int i = 0; i < D->n_quads; ++i)
    if (!mat_ok(D->quad_mat[i]) || D->mat_type[D->quad_mat[i]] == PRDPT_MAT_DIELECTRIC)
      return fail(PRDPT_E_SCENE, "quad material must be diffuse or emissive");
  if (D->n_meshes) {
    if (D->mesh_offset[0] != 0 || D->mesh_offset[D->n_meshes] != D->n_triangles)
      return fail(PRDPT_E_SCENE, "mesh offsets must start at 0 and end at n_triangles");
    for (int m = 0; m < D->n_meshes; ++m) {
      if (D->mesh_offset[m + 1] < D->mesh_offset[m]) return fail(PRDPT_E_SCENE, "mesh offsets decrease");
      if (!mat_ok(D->mesh_mat[m]) || D->mat_type[D->mesh_mat[m]] != PRDPT_MAT_DIFFUSE)
        return fail(PRDPT_E_SCENE, "mesh material must be diffuse");
    }
  } else if (D->n_triangles) {
    return fail(PRDPT_E_SCENE, "triangles without meshes");
  }
  // ---- header ----
  hs = HostScene{};
  SceneHdr& h = hs.hdr;
  std::memcpy(h.eye, D->eye, 12);
  std::memcpy(h.fwd, D->fwd, 12);
  std::memcpy(h.right, D->right, 12);
  std::memcpy(h.up, D->up, 12);
  std::memcpy(h.env, D->env, 12);
  h.W = D->width; h.H = D->height; h.spp = D->spp; h.B = D->max_bounces;
  h.pixel_center = D->pixel_center ? 1 : 0;
  h.n_mat = D->n_materials; h.n_sph = D->n_spheres; h.n_quad = D->n_quads;
  h.n_pl = D->n_point_lights; h.n_param = D->n_params; h.n_tri = D->n_triangles;
  h.tri_id_base = D->n_spheres + D->n_quads;
  for (int i = 0; i < h.n_mat; ++i) {
    h.mat_type[i] = D->mat_type[i];
    for (int c = 0; c < 3; ++c) h.mat_rgb[i][c] = D->mat_rgb[3 * i + c];
    h.mat_ior[i] = D->mat_ior[i];
    if (h.mat_type[i] == PRDPT_MAT_DIELECTRIC) {
      if (!(h.mat_ior[i] > 0.0f) || !std::isfinite(h.mat_ior[i]))
        return fail(PRDPT_E_SCENE, "dielectric ior must be finite and > 0");
      // a dielectric has no colour: its first channel carries 1/ior, the
      // index ratio of a ray entering the body (colour bindings of a
      // dielectric are refused below)
      h.mat_rgb[i][0] = 1.0f / h.mat_ior[i];
    }
  }
  // multiplying by the inverse of a power-of-two size is exact
  h.inv_w = (h.W & (h.W - 1)) == 0 ? 1.0f / (float)h.W : 0.0f;
  h.inv_h = (h.H & (h.H - 1)) == 0 ? 1.0f / (float)h.H : 0.0f;
  h.tile_log2 = render_tile_log2(h.W, h.H, h.spp);
  for (int i = 0; i < h.n_sph; ++i) {
    for (int c = 0; c < 4; ++c) h.sph[i][c] = D->spheres[4 * i + c];
    h.sph_mat[i] = D->sphere_mat[i];
  }
  h.n_area = 0;
  for (int i = 0; i < h.n_quad; ++i) {
    for (int c = 0; c < 9; ++c) h.quad[i][c] = D->quads[9 * i + c];
    quad_frame_host(h.quad[i], h.quad_n[i], h.quad_nu[i]);
    if (!(h.quad_n[i][3] > 0.0f) || !std::isfinite(h.quad_n[i][3]))
      return fail(PRDPT_E_SCENE, "quad edges must span a parallelogram");
    h.quad_lo[i] = quad_neg_limit_host(h.quad_n[i][3]);
    h.quad_mat[i] = D->quad_mat[i];
    if (h.mat_type[h.quad_mat[i]] == PRDPT_MAT_EMISSIVE) h.area_quad[h.n_area++] = i;
  }
  for (int i = 0; i < h.n_pl; ++i)
    for (int c = 0; c < 6; ++c) h.pl[i][c] = D->point_lights[6 * i + c];
  if (D->mesh_rotation)
    for (int i = 0; i < 3 * D->n_meshes; ++i)
      if (!std::isfinite(D->mesh_rotation[i])) return fail(PRDPT_E_SCENE, "mesh rotation not finite");
  // ---- instances: meshes with a binding, a non-zero translation or a non-zero
  //      rotation get their own BVH; all other meshes share one static BVH ----
  std::vector<int> mesh_inst(D->n_meshes, -1);
  std::vector<char> bound(D->n_meshes, 0);
  for (int j = 0; j < D->n_params; ++j) {
    const int kind = D->bindings[3 * j], idx = D->bindings[3 * j + 1], comp = D->bindings[3 * j + 2];
    const int lim = kind == PRDPT_BIND_SPHERE ? D->n_spheres : kind == PRDPT_BIND_QUAD ? D->n_quads
                    : kind == PRDPT_BIND_MESH ? D->n_meshes : kind == PRDPT_BIND_PLIGHT ? D->n_point_lights
                    : kind == PRDPT_BIND_ALBEDO ? D->n_materials
                    : kind == PRDPT_BIND_MESH_ROT ? D->n_meshes : -1;
    if (lim < 0 || idx < 0 || idx >= lim || comp < 0 || comp > 2) {
      return fail(PRDPT_E_SCENE, "bad parameter binding");
    }
    for (int i = 0; i < j; ++i)
      if (D->bindings[3 * i] == kind && D->bindings[3 * i + 1] == idx && D->bindings[3 * i + 2] == comp) {
        return fail(PRDPT_E_SCENE, "a field is bound twice");
      }
    if (kind == PRDPT_BIND_ALBEDO && D->mat_type[idx] == PRDPT_MAT_DIELECTRIC) {
      return fail(PRDPT_E_SCENE, "a dielectric material has no colour to bind");
    }
    if (kind == PRDPT_BIND_MESH || kind == PRDPT_BIND_MESH_ROT) bound[idx] = 1;
    if (kind == PRDPT_BIND_MESH_ROT) h.has_rot = 1;
  }
  int n_inst = 0;
  int static_inst = -1;
  for (int m = 0; m < D->n_meshes; ++m) {
    const float* t = D->mesh_translation + 3 * m;
    const float* a = D->mesh_rotation ? D->mesh_rotation + 3 * m : nullptr;
    const bool rotated = a && (a[0] != 0.0f || a[1] != 0.0f || a[2] != 0.0f);
    if (rotated) h.has_rot = 1;
    const bool own = bound[m] || rotated || t[0] != 0.0f || t[1] != 0.0f || t[2] != 0.0f;
    if (own) {
      mesh_inst[m] = n_inst++;
    } else {
      if (static_inst < 0) static_inst = n_inst++;
      mesh_inst[m] = static_inst;
    }
  }
  if (n_inst > PRDPT_MAX_INSTANCES) {
    return fail(PRDPT_E_SCENE, "too many mesh instances");
  }
  h.n_inst = n_inst;
  for (int j = 0; j < D->n_params; ++j) {
    h.bind_kind[j] = D->bindings[3 * j];
    const bool on_mesh = h.bind_kind[j] == PRDPT_BIND_MESH || h.bind_kind[j] == PRDPT_BIND_MESH_ROT;
    h.bind_index[j] = on_mesh ? mesh_inst[D->bindings[3 * j + 1]] : D->bindings[3 * j + 1];
    h.bind_comp[j] = D->bindings[3 * j + 2];
  }
  std::vector<int32_t> tri_mat(D->n_triangles);
  std::vector<std::vector<int32_t>> lists(n_inst);
  for (int m = 0; m < D->n_meshes; ++m) {
    for (int t = D->mesh_offset[m]; t < D->mesh_offset[m + 1]; ++t) {
      tri_mat[t] = D->mesh_mat[m];
      lists[mesh_inst[m]].push_back(t);
    }
    for (int c = 0; c < 3; ++c) {
      h.inst_xlate[mesh_inst[m]][c] = D->mesh_translation[3 * m + c];
      h.inst_ang[mesh_inst[m]][c] = D->mesh_rotation ? D->mesh_rotation[3 * m + c] : 0.0f;
    }
  }
  for (int i = 0; i < PRDPT_MAX_INSTANCES; ++i) euler_rotation_host(h.inst_ang[i], h.inst_rot[i]);
  std::vector<Node>& nodes = hs.nodes;
  std::vector<Tri>& tris = hs.tris;
  tris.reserve(D->n_triangles);
  for (int i = 0; i < n_inst; ++i) {
    const size_t tri_begin = tris.size();
    BvhOut b = build_bvh(D->triangles, tri_mat.data(), lists[i].data(), (int)lists[i].size(),
                         h.tri_id_base, nodes, tris);
    for (size_t t = tri_begin; t < tris.size(); ++t) tris[t].inst = i;
    if (b.root == -2) {
      return fail(PRDPT_E_SCENE, "mesh instance too large for the BVH depth bound");
    }
    h.inst_root[i] = b.root;
    hs.bvh_depth = std::max(hs.bvh_depth, b.depth);
  }
  if (nodes.size() >= (1u << 24)) {
    return fail(PRDPT_E_SCENE, "too many BVH nodes (at most 2^24)");
  }
  if (hs.bvh_depth > kMaxDepth4) {
    return fail(PRDPT_E_SCENE, "BVH deeper than the traversal stack");
  }
  // the traversal's leaf phase holds at most kLeafMax triangles per lane
  for (const Node& nd : nodes)
    for (int c = 0; c < 4; ++c) {
      const int32_t r = nd.ref[c];
      if (r < 0 && r != kEmptyChild && (~r & 7) + 1 > kLeafMax) {
        return fail(PRDPT_E_SCENE, "BVH leaf larger than the traversal's leaf bound");
      }
    }
  // every scene triangle lands in exactly one leaf: a permutation
  hs.tri_slot.assign(tris.size(), -1);
  for (size_t t = 0; t < tris.size(); ++t) {
    const int64_t i = (int64_t)tris[t].id - h.tri_id_base;
    if (i < 0 || i >= (int64_t)tris.size() || hs.tri_slot[i] >= 0) {
      return fail(PRDPT_E_SCENE, "BVH triangles are not a permutation of the scene's");
    }
    hs.tri_slot[i] = (int32_t)t;
  }
  hs.footprint = sizeof(SceneHdr) + nodes.size() * sizeof(Node) + tris.size() * sizeof(Tri) +
                 tris.size() * sizeof(int32_t) +
                 (size_t)render_tiles(h.W, h.H, h.tile_log2) * (sizeof(float) + sizeof(int));
  return PRDPT_OK;
}

// Admit (context HBM budget) and upload a host-built scene.
int prdpt::upload_scene(prdpt_ctx* ctx, const HostScene& hs, prdpt_scene** out) {
  prdpt_scene* s = new prdpt_scene();
  s->ctx = ctx;
  s->hdr = hs.hdr;
  s->bvh_depth = hs.bvh_depth;
  s->n_nodes = (int)hs.nodes.size();
  s->n_tris = (int)hs.tris.size();
  s->footprint = hs.footprint;
  const SceneHdr& h = hs.hdr;
  const std::vector<Node>& nodes = hs.nodes;
  const std::vector<Tri>& tris = hs.tris;
  // ---- admission and upload ----
  std::lock_guard<std::mutex> g(ctx->mu);
  if (ctx->budget && ctx->resident + s->footprint > ctx->budget) {
    delete s;
    return fail(PRDPT_E_ADMISSION, "scene exceeds the context's HBM budget");
  }
  if (hipSetDevice(ctx->device) != hipSuccess) {
    delete s;
    return fail(PRDPT_E_HIP, "hipSetDevice failed");
  }
  s->n_tiles = render_tiles(h.W, h.H, h.tile_log2);
  auto release = [&]() {
    if (s->d_hdr) hipFree(s->d_hdr);
    if (s->d_nodes) hipFree(s->d_nodes);
    if (s->d_tris) hipFree(s->d_tris);
    if (s->d_tri_slot) hipFree(s->d_tri_slot);
    if (s->d_tile_cost) hipFree(s->d_tile_cost);
    if (s->d_tile_order) hipFree(s->d_tile_order);
    delete s;
  };
  bool ok = dev_malloc((void**)&s->d_hdr, sizeof(SceneHdr)) == hipSuccess;
  ok = ok && dev_malloc((void**)&s->d_nodes, std::max<size_t>(1, nodes.size()) * sizeof(Node)) == hipSuccess;
  ok = ok && dev_malloc((void**)&s->d_tris, std::max<size_t>(1, tris.size()) * sizeof(Tri)) == hipSuccess;
  ok = ok && dev_malloc((void**)&s->d_tri_slot, std::max<size_t>(1, tris.size()) * sizeof(int32_t)) == hipSuccess;
  ok = ok && dev_malloc((void**)&s->d_tile_cost, s->n_tiles * sizeof(float)) == hipSuccess;
  ok = ok && dev_malloc((void**)&s->d_tile_order, s->n_tiles * sizeof(int)) == hipSuccess;
  if (!ok) {
    release();
    return fail(PRDPT_E_NOMEM, "device allocation of the scene failed");
  }
  std::vector<int> order(s->n_tiles);
  for (int i = 0; i < s->n_tiles; ++i) order[i] = i;
  const std::vector<float> cost(s->n_tiles, 0.0f);
  ok = hipMemcpy(s->d_hdr, &h, sizeof(SceneHdr), hipMemcpyHostToDevice) == hipSuccess;
  if (ok && !nodes.empty())
    ok = hipMemcpy(s->d_nodes, nodes.data(), nodes.size() * sizeof(Node), hipMemcpyHostToDevice) == hipSuccess;
  if (ok && !tris.empty())
    ok = hipMemcpy(s->d_tris, tris.data(), tris.size() * sizeof(Tri), hipMemcpyHostToDevice) == hipSuccess;
  if (ok && !tris.empty())
    ok = hipMemcpy(s->d_tri_slot, hs.tri_slot.data(), tris.size() * sizeof(int32_t),
                   hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(s->d_tile_order, order.data(), s->n_tiles * sizeof(int), hipMemcpyHostToDevice) ==
                 hipSuccess;
  ok = ok && hipMemcpy(s->d_tile_cost, cost.data(), s->n_tiles * sizeof(float), hipMemcpyHostToDevice) ==
                 hipSuccess;
  if (!ok) {
    release();
    return fail(PRDPT_E_HIP, "scene upload failed");
  }
  ctx->resident += s->footprint;
  ctx->n_scenes++;
  *out = s;
  return PRDPT_OK;
}

extern "C" {

int prdpt_scene_create(prdpt_ctx* ctx, const prdpt_scene_desc* D, prdpt_scene** out,
                       size_t* footprint_bytes) {
  if (!ctx || !D || !out) return fail(PRDPT_E_ARG, "null argument");
  *out = nullptr;
  HostScene hs;
  if (int rc = build_host_scene(D, hs)) return rc;
  if (int rc = upload_scene(ctx, hs, out)) return rc;
  if (footprint_bytes) *footprint_bytes = (*out)->footprint;
  return PRDPT_OK;
}

int prdpt_scene_destroy(prdpt_scene* s) {
  if (!s) return fail(PRDPT_E_ARG, "scene is null");
  prdpt_ctx* ctx = s->ctx;
  std::lock_guard<std::mutex> g(ctx->mu);
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  hipFree(s->d_hdr);
  hipFree(s->d_nodes);
  hipFree(s->d_tris);
  hipFree(s->d_tri_slot);
  hipFree(s->d_tile_cost);
  hipFree(s->d_tile_order);
  ctx->resident -= s->footprint;
  ctx->n_scenes--;
  delete s;
  return PRDPT_OK;
}

int prdpt_scene_info(const prdpt_scene* s, int* width, int* height, int* spp, int* max_bounces,
                     int* n_params) {
  if (!s) return fail(PRDPT_E_ARG, "scene is null");
  if (width) *width = s->hdr.W;
  if (height) *height = s->hdr.H;
  if (spp) *spp = s->hdr.spp;
  if (max_bounces) *max_bounces = s->hdr.B;
  if (n_params) *n_params = s->hdr.n_param;
  return PRDPT_OK;
}

int prdpt_draw_tau(prdpt_ctx* ctx, int est, int d, int P, uint64_t seed, const float* sigma,
                   float* tau_out, double* c_out) {
  if (!ctx || !sigma || !tau_out || !c_out) return fail(PRDPT_E_ARG, "null argument");
  if (d < 1 || d > PRDPT_MAX_PARAMS || P < 1 || P > (1 << 20)) return fail(PRDPT_E_ARG, "bad d or P");
  if (int rc = check_est(est)) return rc;
  for (int j = 0; j < d; ++j)
    if (!(sigma[j] > 0.0f) || !std::isfinite(sigma[j])) return fail(PRDPT_E_ARG, "sigma must be > 0");
  std::lock_guard<std::mutex> g(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->device));
  if (int rc = prepare(ctx, 2 * P, d, 1)) return rc;
  std::vector<float> zero(d, 0.0f);
  if (int rc = upload_vectors(ctx, zero.data(), sigma, d)) return rc;
  HIP_TRY(launch_tau(ctx->stream, est, d, P, seed, ctx->sigma.p, ctx->theta.p, chi_mean(d),
                     std::sqrt(2.0 * M_PI), ctx->tau.p, ctx->c.p, ctx->X.p));
  HIP_TRY(hipMemcpyAsync(tau_out, ctx->tau.p, sizeof(float) * P * d, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipMemcpyAsync(c_out, ctx->c.p, sizeof(double) * P * d, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return PRDPT_OK;
}

int prdpt_render_perturbed(prdpt_scene* s, const float* theta, const float* sigma, int N,
                           uint64_t seed, int est, float* images_out, float* tau_out) {
  if (int rc = check_request(s, theta, sigma, N, true)) return rc;
  if (int rc = check_est(est)) return rc;
  if (!images_out) return fail(PRDPT_E_ARG, "images_out is null");
  prdpt_ctx* ctx = s->ctx;
  const SceneHdr& h = s->hdr;
  const int d = h.n_param, rows = n_draws(est, N);
  std::lock_guard<std::mutex> g(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->device));
  if (int rc = prepare(ctx, N, d, render_tiles(h.W, h.H, h.tile_log2))) return rc;
  if (int rc = upload_vectors(ctx, theta, sigma, d)) return rc;
  HIP_TRY(launch_tau(ctx->stream, est, d, rows, seed, ctx->sigma.p, ctx->theta.p, chi_mean(d),
                     std::sqrt(2.0 * M_PI), ctx->tau.p, ctx->c.p, ctx->X.p));
  HIP_TRY(launch_render(ctx->stream, s->dev(), h.W, h.H, h.tile_log2, ctx->X.p, N, d, kTagPath, seed, nullptr,
                        images_out, nullptr, nullptr, ctx->work.p, s->d_tile_order,
                        s->d_tile_cost, (est & PRDPT_EST_INDEPENDENT) ? 0 : 1, h.has_rot,
                        h.n_sph));
  if (tau_out)
    HIP_TRY(hipMemcpyAsync(tau_out, ctx->tau.p, sizeof(float) * rows * d, hipMemcpyDeviceToHost,
                           ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return PRDPT_OK;
}

int prdpt_render_reference(prdpt_scene* s, const float* X, uint64_t seed, float* image_out) {
  if (!s || !X || !image_out) return fail(PRDPT_E_ARG, "null argument");
  prdpt_ctx* ctx = s->ctx;
  const SceneHdr& h = s->hdr;
  const int d = h.n_param;
  std::lock_guard<std::mutex> g(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->device));
  if (int rc = prepare(ctx, 2, d, render_tiles(h.W, h.H, h.tile_log2))) return rc;
  HIP_TRY(hipMemcpyAsync(ctx->X.p, X, sizeof(float) * d, hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(launch_render(ctx->stream, s->dev(), h.W, h.H, h.tile_log2, ctx->X.p, 1, d, kTagRef, seed, nullptr,
                        image_out, nullptr, nullptr, ctx->work.p, s->d_tile_order,
                        s->d_tile_cost, 1, h.has_rot, h.n_sph));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return PRDPT_OK;
}

int prdpt_grad_estimate(prdpt_scene* s, const float* ref, const float* theta, const float* sigma,
                        int N, uint64_t seed, int est, double* grad_out, double* loss_out,
                        double* losses_out) {
  if (int rc = check_request(s, theta, sigma, N, true)) return rc;
  if (int rc = check_est(est)) return rc;
  if (!ref || !grad_out) return fail(PRDPT_E_ARG, "ref/grad_out is null");
  prdpt_ctx* ctx = s->ctx;
  const int d = s->hdr.n_param;
  std::lock_guard<std::mutex> g(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->device));
  if (int rc = prepare(ctx, N, d, render_tiles(s->hdr.W, s->hdr.H, s->hdr.tile_log2))) return rc;
  // one pinned upload of [theta | sigma], one pinned download of
  // [grad | loss | losses]
  const size_t n_in = 2 * (size_t)d, n_out = (size_t)d + 1 + (size_t)N;
  if (int rc = ensure(ctx, ctx->vin, n_in)) return rc;
  if (int rc = ensure(ctx, ctx->vout, n_out)) return rc;
  if (int rc = ensure_pinned(ctx, ctx->h_vin, ctx->h_vin_n, n_in)) return rc;
  if (int rc = ensure_pinned(ctx, ctx->h_vout, ctx->h_vout_n, n_out)) return rc;
  std::memcpy(ctx->h_vin, theta, sizeof(float) * d);
  std::memcpy(ctx->h_vin + d, sigma, sizeof(float) * d);
  HIP_TRY(hipMemcpyAsync(ctx->vin.p, ctx->h_vin, sizeof(float) * n_in, hipMemcpyHostToDevice,
                         ctx->stream));
  double* out = ctx->vout.p;
  if (int rc = enqueue_estimate(s, ref, ctx->vin.p, ctx->vin.p + d, N, seed, est, out, out + d,
                                out + d + 1, nullptr))
    return rc;
  HIP_TRY(hipMemcpyAsync(ctx->h_vout, out, sizeof(double) * n_out, hipMemcpyDeviceToHost,
                         ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  std::memcpy(grad_out, ctx->h_vout, sizeof(double) * d);
  if (loss_out) *loss_out = ctx->h_vout[d];
  if (losses_out) std::memcpy(losses_out, ctx->h_vout + d + 1, sizeof(double) * N);
  return PRDPT_OK;
}

int prdpt_grad_estimate_dp(prdpt_scene* s, const float* ref, const float* theta, const float* sigma,
                           int N, uint64_t seed, int edge_samples, double* grad_out,
                           double* loss_out, double* losses_out) {
  if (int rc = check_request(s, theta, sigma, N, true)) return rc;
  if (!ref || !grad_out) return fail(PRDPT_E_ARG, "ref/grad_out is null");
  if (edge_samples < 1 || edge_samples > (1 << 24))
    return fail(PRDPT_E_ARG, "edge_samples must be in 1..2^24");
  const SceneHdr& h = s->hdr;
  // the differentiable renderer: one diffuse sphere whose centre is bound,
  // one diffuse quad (the ground), one point light, no meshes, no bounces
  bool ok = h.n_sph == 1 && h.n_quad == 1 && h.n_inst == 0 && h.n_tri == 0 && h.n_pl == 1 &&
            h.B == 0 && h.mat_type[h.sph_mat[0]] == PRDPT_MAT_DIFFUSE &&
            h.mat_type[h.quad_mat[0]] == PRDPT_MAT_DIFFUSE && h.n_param >= 1 && h.n_param <= 3;
  for (int j = 0; ok && j < h.n_param; ++j)
    ok = h.bind_kind[j] == PRDPT_BIND_SPHERE && h.bind_index[j] == 0;
  if (!ok)
    return fail(PRDPT_E_SCENE, "Eq. 9 needs one diffuse sphere (its centre bound) over one diffuse "
                               "quad under one point light, direct light only");
  prdpt_ctx* ctx = s->ctx;
  const int d = h.n_param, P = N / 2;
  const size_t npix = (size_t)h.W * h.H;
  const int bi = dp_interior_blocks(h.W, h.H), be = dp_edge_blocks(edge_samples);
  std::lock_guard<std::mutex> g(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->device));
  if (int rc = prepare(ctx, N, d, render_tiles(h.W, h.H, h.tile_log2))) return rc;
  if (int rc = ensure(ctx, ctx->images, (size_t)N * npix * 3)) return rc;
  if (int rc = ensure(ctx, ctx->dp_partial, (size_t)N * (bi + be) * 3)) return rc;
  if (int rc = upload_vectors(ctx, theta, sigma, d)) return rc;
  HIP_TRY(launch_tau(ctx->stream, PRDPT_EST_GAUSS, d, P, seed, ctx->sigma.p, ctx->theta.p,
                     chi_mean(d), std::sqrt(2.0 * M_PI), ctx->tau.p, ctx->c.p, ctx->X.p));
  HIP_TRY(timed_render(ctx, s, ctx->X.p, N, d, kTagPath, seed, ref, ctx->images.p, ctx->partial.p, 1,
                       ctx->work.p));
  HIP_TRY(launch_losses(ctx->stream, ctx->partial.p, render_tiles(h.W, h.H, h.tile_log2), N, (int)npix,
                        ctx->losses.p));
  double* pin = ctx->dp_partial.p;
  double* pedge = pin + (size_t)N * bi * 3;
  HIP_TRY(launch_dp(ctx->stream, s->d_hdr, h.W, h.H, ctx->X.p, N, d, seed, ctx->images.p, ref,
                    edge_samples, pin, pedge, ctx->losses.p, ctx->grad.p, ctx->loss.p));
  HIP_TRY(hipMemcpyAsync(grad_out, ctx->grad.p, sizeof(double) * d, hipMemcpyDeviceToHost, ctx->stream));
  double q = 0.0;
  HIP_TRY(hipMemcpyAsync(&q, ctx->loss.p, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  if (losses_out)
    HIP_TRY(hipMemcpyAsync(losses_out, ctx->losses.p, sizeof(double) * N, hipMemcpyDeviceToHost,
                           ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (loss_out) *loss_out = q;
  return PRDPT_OK;
}

int prdpt_smoothed_loss(prdpt_scene* s, const float* ref, const float* theta, const float* sigma,
                        int N, uint64_t seed, double* loss_out) {
  if (!loss_out) return fail(PRDPT_E_ARG, "loss_out is null");
  if (int rc = check_request(s, theta, sigma, N, true)) return rc;
  if (!ref) return fail(PRDPT_E_ARG, "ref is null");
  prdpt_ctx* ctx = s->ctx;
  const int d = s->hdr.n_param;
  std::lock_guard<std::mutex> g(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->device));
  if (int rc = prepare(ctx, N, d, render_tiles(s->hdr.W, s->hdr.H, s->hdr.tile_log2))) return rc;
  if (int rc = upload_vectors(ctx, theta, sigma, d)) return rc;
  if (int rc = enqueue_estimate(s, ref, ctx->theta.p, ctx->sigma.p, N, seed, PRDPT_EST_GAUSS,
                                ctx->grad.p, ctx->loss.p, nullptr, nullptr))
    return rc;
  HIP_TRY(hipMemcpyAsync(loss_out, ctx->loss.p, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return PRDPT_OK;
}

int prdpt_grad_estimate_async(prdpt_scene* s, const float* ref_dev, const float* theta_dev,
                              const float* sigma_dev, int N, uint64_t seed, int est,
                              double* grad_dev, double* loss_dev, double* losses_dev,
                              double* c_dev) {
  if (int rc = check_request(s, theta_dev, sigma_dev, N, false)) return rc;
  if (int rc = check_est(est)) return rc;
  if (!ref_dev || !grad_dev || !loss_dev) return fail(PRDPT_E_ARG, "null device pointer");
  prdpt_ctx* ctx = s->ctx;
  std::lock_guard<std::mutex> g(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->device));
  return enqueue_estimate(s, ref_dev, theta_dev, sigma_dev, N, seed, est, grad_dev, loss_dev,
                          losses_dev, c_dev);
}

int prdpt_grad_estimate_noalloc(prdpt_scene* s, const float* ref_dev, const float* theta_dev,
                                const float* sigma_dev, int N, uint64_t seed, int est,
                                double* grad_dev, double* loss_dev, double* losses_dev,
                                double* c_dev) {
  if (int rc = check_request(s, theta_dev, sigma_dev, N, false)) return rc;
  if (int rc = check_est(est)) return rc;
  if (!ref_dev || !grad_dev || !loss_dev) return fail(PRDPT_E_ARG, "null device pointer");
  prdpt_ctx* ctx = s->ctx;
  const SceneHdr& h = s->hdr;
  const size_t d = (size_t)h.n_param, rows = (size_t)n_draws(est, N);
  const size_t n_tiles = (size_t)render_tiles(h.W, h.H, h.tile_log2);
  // the estimate's arrays, each at a 256-byte boundary of the scratch array
  size_t used = 0;
  auto take = [&](size_t bytes) {
    const size_t at = used;
    used += (bytes + 255) & ~(size_t)255;
    return at;
  };
  const size_t oX = take((size_t)N * d * sizeof(float));
  const size_t otau = take(rows * d * sizeof(float));
  const size_t oc = c_dev ? 0 : take(rows * d * sizeof(double));
  const size_t opart = take((size_t)N * n_tiles * sizeof(float));
  const size_t oL = losses_dev ? 0 : take((size_t)N * sizeof(double));
  const size_t owork = take(sizeof(int));
  if (used > (size_t)PRDPT_NOALLOC_SCRATCH_BYTES)
    return fail(PRDPT_E_ARG, "the request needs " + std::to_string(used) +
                                 " bytes of scratch, more than the allocation-free estimate's " +
                                 std::to_string((size_t)PRDPT_NOALLOC_SCRATCH_BYTES));
  std::lock_guard<std::mutex> g(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->device));
  if (!ctx->scratch)
    return fail(PRDPT_E_HIP, std::string("scratch array unavailable: ") +
                                 hipGetErrorString(ctx->scratch_status));
  char* base = static_cast<char*>(ctx->scratch);
  const EstimateBufs b{reinterpret_cast<float*>(base + oX), reinterpret_cast<float*>(base + otau),
                       c_dev ? nullptr : reinterpret_cast<double*>(base + oc),
                       reinterpret_cast<float*>(base + opart),
                       losses_dev ? nullptr : reinterpret_cast<double*>(base + oL),
                       reinterpret_cast<int*>(base + owork)};
  return enqueue_into(s, ref_dev, theta_dev, sigma_dev, N, seed, est, grad_dev, loss_dev,
                      losses_dev, c_dev, b, false);
}

int prdpt_combine_async(prdpt_ctx* ctx, int rows, int d, const double* c_dev,
                        const double* losses_dev, const double* scale_dev, double* grad_dev,
                        int est) {
  if (!ctx || !c_dev || !losses_dev || !grad_dev) return fail(PRDPT_E_ARG, "null argument");
  if (rows < 1 || rows > (1 << 20) || d < 1 || d > PRDPT_MAX_PARAMS)
    return fail(PRDPT_E_ARG, "rows must be in 1..2^20 and d in 1..PRDPT_MAX_PARAMS");
  if (int rc = check_est(est)) return rc;
  std::lock_guard<std::mutex> g(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(launch_combine(ctx->stream, rows, d, (est & PRDPT_EST_INDEPENDENT) ? 1 : 0, c_dev,
                         losses_dev, scale_dev, grad_dev, nullptr));
  return PRDPT_OK;
}

int prdpt_ctx_set_timing(prdpt_ctx* ctx, int enable) {
  if (!ctx) return fail(PRDPT_E_ARG, "ctx is null");
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->timing = enable != 0;
  return PRDPT_OK;
}

int prdpt_ctx_read_timing(prdpt_ctx* ctx, double* total_ms, int64_t* launches) {
  if (!ctx || !total_ms || !launches) return fail(PRDPT_E_ARG, "null argument");
  std::lock_guard<std::mutex> g(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->device));
  for (auto& pr : ctx->pending) {
    HIP_TRY(hipEventSynchronize(pr.second));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
    ctx->timed_ms += ms;
    ctx->timed_launches += 1;
    ctx->pool.push_back(pr.first);
    ctx->pool.push_back(pr.second);
  }
  ctx->pending.clear();
  *total_ms = ctx->timed_ms;
  *launches = ctx->timed_launches;
  ctx->timed_ms = 0.0;
  ctx->timed_launches = 0;
  return PRDPT_OK;
}

int prdpt_traversal_counts(prdpt_scene* s, const float* theta, const float* sigma, int N,
                           uint64_t seed, int est, uint64_t* counts) {
  if (int rc = check_request(s, theta, sigma, N, true)) return rc;
  if (int rc = check_est(est)) return rc;
  if (!counts) return fail(PRDPT_E_ARG, "counts is null");
  prdpt_ctx* ctx = s->ctx;
  const SceneHdr& h = s->hdr;
  const int d = h.n_param, rows = n_draws(est, N);
  std::lock_guard<std::mutex> g(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->device));
  if (int rc = prepare(ctx, N, d, render_tiles(h.W, h.H, h.tile_log2))) return rc;
  if (int rc = ensure(ctx, ctx->counters, 10)) return rc;
  if (int rc = upload_vectors(ctx, theta, sigma, d)) return rc;
  HIP_TRY(hipMemsetAsync(ctx->counters.p, 0, 10 * sizeof(unsigned long long), ctx->stream));
  HIP_TRY(launch_tau(ctx->stream, est, d, rows, seed, ctx->sigma.p, ctx->theta.p, chi_mean(d),
                     std::sqrt(2.0 * M_PI), ctx->tau.p, ctx->c.p, ctx->X.p));
  HIP_TRY(launch_render(ctx->stream, s->dev(), h.W, h.H, h.tile_log2, ctx->X.p, N, d, kTagPath, seed, nullptr,
                        nullptr, nullptr, ctx->counters.p, ctx->work.p, s->d_tile_order,
                        nullptr, (est & PRDPT_EST_INDEPENDENT) ? 0 : 1, s->hdr.has_rot,
                        s->hdr.n_sph));
  unsigned long long host[10];
  HIP_TRY(hipMemcpyAsync(host, ctx->counters.p, sizeof(host), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < 10; ++i) counts[i] = host[i];
  return PRDPT_OK;
}

int prdpt_copy_probe(prdpt_ctx* ctx, const void* src, void* dst, size_t bytes, int iters,
                     double* ms_per_copy) {
  if (!ctx || !src || !dst || !ms_per_copy || iters < 1) return fail(PRDPT_E_ARG, "bad probe arguments");
  if (bytes == 0 || bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16)
    return fail(PRDPT_E_ARG, "bytes and pointers must be 16-byte aligned and non-zero");
  std::lock_guard<std::mutex> g(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->device));
  hipEvent_t a, b;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  HIP_TRY(launch_copy(ctx->stream, src, dst, bytes / 16));  // warm-up
  HIP_TRY(hipEventRecord(a, ctx->stream));
  for (int i = 0; i < iters; ++i) HIP_TRY(launch_copy(ctx->stream, src, dst, bytes / 16));
  HIP_TRY(hipEventRecord(b, ctx->stream));
  HIP_TRY(hipEventSynchronize(b));
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, a, b));
  hipEventDestroy(a);
  hipEventDestroy(b);
  *ms_per_copy = (double)ms / iters;
  return PRDPT_OK;
}

int prdpt_selftest_math(prdpt_ctx* ctx, uint64_t* mismatches) {
  if (!ctx || !mismatches) return fail(PRDPT_E_ARG, "bad self-test arguments");
  std::lock_guard<std::mutex> g(ctx->mu);
  HIP_TRY(hipSetDevice(ctx->device));
  unsigned long long* d = nullptr;
  if (dev_malloc((void**)&d, 3 * sizeof(unsigned long long)) != hipSuccess)
    return fail(PRDPT_E_NOMEM, "self-test counters");
  hipError_t e = hipMemsetAsync(d, 0, 3 * sizeof(unsigned long long), ctx->stream);
  if (e == hipSuccess) e = launch_math_selftest(ctx->stream, d);
  unsigned long long h[3] = {0, 0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(PRDPT_E_HIP, hipGetErrorString(e));
  for (int i = 0; i < 3; ++i) mismatches[i] = h[i];
  return PRDPT_OK;
}

double prdpt_sigma_schedule(double sigma0, double sigma_end, int t, int T) {
  if (T <= 1) return sigma0;
  return sigma0 + (sigma_end - sigma0) * (double)t / (double)(T - 1);
}

int prdpt_adam_step(int d, double* theta, const double* grad, double* m, double* v, int t,
                    double lr, double beta1, double beta2, double eps) {
  if (d < 1 || !theta || !grad || !m || !v || t < 1) return fail(PRDPT_E_ARG, "bad Adam arguments");
  const double c1 = 1.0 - std::pow(beta1, t), c2 = 1.0 - std::pow(beta2, t);
  for (int j = 0; j < d; ++j) {
    m[j] = beta1 * m[j] + (1.0 - beta1) * grad[j];
    v[j] = beta2 * v[j] + (1.0 - beta2) * grad[j] * grad[j];
    theta[j] -= lr * (m[j] / c1) / (std::sqrt(v[j] / c2) + eps);
  }
  return PRDPT_OK;
}

}  // extern "C"
