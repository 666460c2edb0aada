// Context and scene internals shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "prdpt.h"
#include "prdpt_internal.h"

namespace prdpt {
BvhOut build_bvh(const float* tri9, const int32_t* tri_mat, const int32_t* list, int n,
                 int32_t id_base, std::vector<Node>& nodes, std::vector<Tri>& tris);
// render tiles of an image with tiles of 2^tile_log2 square pixels, and the
// tile size the library chooses for an image (scene constant tile_log2)
int render_tiles(int W, int H, int tile_log2);
int render_tile_log2(int W, int H, int spp);
hipError_t launch_tau(hipStream_t st, int est, int d, int P, uint64_t seed, const float* sigma,
                      const float* theta, double cd, double sqrt2pi, float* tau, double* c, float* X);
hipError_t launch_render(hipStream_t st, const DevScene& sc, int W, int H, int tile_log2,
                         const float* X, int nk,
                         int d, int tag, uint64_t seed, const float* ref, float* img,
                         float* partial, unsigned long long* counters, int* work,
                         const int* order, float* cost, int crn, int rot, int n_sph);
// resident render work-groups for a variant and sphere count (the grid bound)
int render_grid_limit(int rot, int n_sph, int tile_log2);
int batch_grid_limit(int rot, int max_sph);
// Rz(c) Ry(b) Rx(a) of the angles (a, b, c), row-major (the kernels' own formula)
void euler_rotation_host(const float* ang, float* R);
// normal and squared length, unit normal and area of a quad [origin, edge1,
// edge2] (the kernels' operation order)
void quad_frame_host(const float* q, float* n, float* nu);
// largest x whose correctly rounded x / nn is below 0 (nn > 0 finite)
float quad_neg_limit_host(float nn);
// tiles by descending measured render time (no-op for more than 4096 tiles)
hipError_t launch_tile_order(hipStream_t st, const float* cost, int* order, int n_tiles);
hipError_t launch_losses(hipStream_t st, const float* partial, int n_tiles, int N, int npix,
                         double* losses);
// rows = pairs (antithetic) or draws (independent != 0)
hipError_t launch_combine(hipStream_t st, int rows, int d, int independent, const double* c,
                          const double* L, const double* scale, double* grad, double* loss);
// rot != 0: some request's scene has rotated instances; max_sph: the largest
// sphere count of the batch's scenes (sizes the render kernel's dynamic LDS)
hipError_t launch_batch(hipStream_t st, const BatchReq* reqs, BatchMeta* meta, int render_blocks,
                        int rot, int max_sph, float* tau, double* c, float* X,
                        float* partial, double* losses, double* grads, double* loss);
hipError_t launch_copy(hipStream_t st, const void* src, void* dst, size_t n16);
// exhaustive check of the render kernel's fast correctly rounded reciprocal
// and square root (exact_math.h): adds the mismatch counts to bad[0..2]
hipError_t launch_math_selftest(hipStream_t st, unsigned long long* bad);
// Eq. 9: interior and edge derivative terms of N renders weighted by their
// (I - R), reduced to the gradient and the mean loss; pin/pedge hold
// N x dp_interior_blocks / dp_edge_blocks rows of 3 doubles
int dp_interior_blocks(int W, int H);
int dp_edge_blocks(int M);
hipError_t launch_dp(hipStream_t st, const SceneHdr* hdr, int W, int H, const float* X, int N, int d,
                     uint64_t seed, const float* img, const float* ref, int M, double* pin,
                     double* pedge, const double* losses, double* grad, double* loss);
// device address of the current device's copy of the allocation-free
// estimate's scratch array (PRDPT_NOALLOC_SCRATCH_BYTES), looked up once per
// device; `device` must be current
hipError_t noalloc_scratch(int device, void** out);

// records `msg` as the calling thread's last error and returns `code`
int fail(int code, const std::string& msg);
// every device and pinned host allocation of the library goes through these
// two (prdpt_debug_fail_allocations makes them fail on request)
hipError_t dev_malloc(void** p, size_t bytes);
hipError_t pinned_malloc(void** p, size_t bytes);

// Mean of the chi distribution with d degrees of freedom (the IS weight constant):
// C_1 = sqrt(2/pi), C_{k+1} = k / C_k.
inline double chi_mean(int d) {
  double c = std::sqrt(2.0 / M_PI);
  for (int k = 1; k < d; ++k) c = (double)k / c;
  return c;
}

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
};

// Device and pinned buffers, graph and launch configuration of the batched form.
struct BatchState {
  hipStream_t stream = nullptr;  // own non-blocking stream (capturable)
  hipEvent_t ready = nullptr;    // orders the batch stream after the context stream
  int n_cu = 0;
  int blocks_per_cu = 0, tiles_per_item = 1, use_graph = 1;  // 0: as many as are resident
  size_t cap_req = 0, cap_pairs = 0, cap_rows = 0, cap_partial = 0;
  BatchReq* d_reqs = nullptr;
  BatchMeta* d_meta = nullptr;
  float* d_tau = nullptr;
  double* d_c = nullptr;
  float* d_X = nullptr;
  float* d_partial = nullptr;
  double* d_losses = nullptr;
  double* d_grads = nullptr;
  double* d_loss = nullptr;
  BatchReq* h_reqs = nullptr;      // pinned
  BatchMeta* h_meta = nullptr;     // pinned
  double* h_grads = nullptr;       // pinned
  double* h_loss = nullptr;        // pinned
  double* h_losses = nullptr;      // pinned
  hipGraphExec_t exec = nullptr;
  int graph_blocks = 0;
  int graph_rot = 0;  // render variant captured in the graph
  int graph_sph = 0;  // sphere count its dynamic LDS was sized for
};

void batch_release(BatchState& b);

// A scene validated and built on the host (header, BVH nodes, triangles).
struct HostScene {
  SceneHdr hdr{};
  std::vector<Node> nodes;
  std::vector<Tri> tris;
  std::vector<int32_t> tri_slot;  // index in tris of each scene triangle
  int bvh_depth = 0;
  size_t footprint = 0;
};
}  // namespace prdpt

struct prdpt_ctx;
struct prdpt_scene;
namespace prdpt {
int build_host_scene(const prdpt_scene_desc* D, HostScene& hs);
int upload_scene(prdpt_ctx* ctx, const HostScene& hs, prdpt_scene** out);
int ensure_batch(prdpt_ctx* ctx, BatchState& b, size_t n_req, size_t pairs, size_t rows,
                 size_t partial);
int batch_enqueue(prdpt_ctx* ctx, BatchState& b, prdpt_request* reqs, int n, std::vector<int>& ok,
                  hipEvent_t t0, hipEvent_t t1);
void batch_collect(BatchState& b, prdpt_request* reqs, const std::vector<int>& ok);
}  // namespace prdpt

struct prdpt_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;
  size_t resident = 0;
  int n_scenes = 0;
  std::mutex mu;
  prdpt::DevBuf<float> X, tau, partial, theta, sigma;
  prdpt::DevBuf<float> images;          // Eq. 9: the N rendered images
  prdpt::DevBuf<double> dp_partial;     // Eq. 9: per-block derivative terms
  prdpt::DevBuf<double> c, losses, grad, loss;
  prdpt::DevBuf<unsigned long long> counters;
  prdpt::DevBuf<int> work;  // work counter of the persistent render kernel
  // this device's scratch array of prdpt_grad_estimate_noalloc (null: lookup failed)
  void* scratch = nullptr;
  hipError_t scratch_status = hipSuccess;
  // the synchronous estimate's inputs [theta | sigma] and outputs
  // [grad | loss | losses], each moved by one copy through pinned host memory
  prdpt::DevBuf<float> vin;
  prdpt::DevBuf<double> vout;
  float* h_vin = nullptr;   // pinned
  double* h_vout = nullptr; // pinned
  size_t h_vin_n = 0, h_vout_n = 0;
  // optional timing of the fused render kernel (events on the context stream)
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  std::vector<hipEvent_t> pool;
  double timed_ms = 0.0;
  int64_t timed_launches = 0;
  prdpt::BatchState batch;
};

struct prdpt_scene {
  prdpt_ctx* ctx = nullptr;
  prdpt::SceneHdr hdr{};
  prdpt::SceneHdr* d_hdr = nullptr;
  prdpt::Node* d_nodes = nullptr;
  prdpt::Tri* d_tris = nullptr;
  int32_t* d_tri_slot = nullptr;
  float* d_tile_cost = nullptr;  // last measured render time per pixel tile
  int* d_tile_order = nullptr;   // tiles by descending cost (render order)
  int n_tiles = 0;
  size_t footprint = 0;
  int n_nodes = 0, n_tris = 0, bvh_depth = 0;
  prdpt::DevScene dev() const { return prdpt::DevScene{d_hdr, d_nodes, d_tris, d_tri_slot}; }
};

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return ::prdpt::fail(PRDPT_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
