// Host-side checks of the library under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_host_sanitizers.py; runs
// without a GPU).  Exercises scene validation and the BVH builder on random,
// degenerate and deep triangle sets, checks the built trees' invariants (every
// triangle in exactly one leaf, padded leaf boxes containing their triangles,
// 4-wide depth within the traversal stack bound), every entry point's argument
// checks, the host optimiser step, and context creation without a device.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <random>
#include <vector>

#include "ctx_internal.h"

using namespace prdpt;

static int g_failures = 0;
#define CHECK(c)                                                             \
  do {                                                                       \
    if (!(c)) {                                                              \
      std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c);   \
      ++g_failures;                                                          \
    }                                                                        \
  } while (0)

struct SceneArrays {
  std::vector<int32_t> mat_type{0};
  std::vector<float> mat_rgb{0.5f, 0.5f, 0.5f};
  std::vector<float> mat_ior{1.0f};
  std::vector<float> tris;
  std::vector<int32_t> mesh_off{0, 0};
  std::vector<int32_t> mesh_mat{0};
  std::vector<float> mesh_xlate{0.0f, 0.0f, 0.0f};
  std::vector<int32_t> bindings{2, 0, 0};
  prdpt_scene_desc desc() {
    prdpt_scene_desc d{};
    float eye[3] = {0, 0, 5}, fwd[3] = {0, 0, -1}, right[3] = {0.4f, 0, 0}, up[3] = {0, 0.4f, 0};
    for (int i = 0; i < 3; ++i) {
      d.eye[i] = eye[i];
      d.fwd[i] = fwd[i];
      d.right[i] = right[i];
      d.up[i] = up[i];
    }
    d.width = 16;
    d.height = 12;
    d.spp = 1;
    d.max_bounces = 1;
    d.n_materials = 1;
    d.mat_type = mat_type.data();
    d.mat_rgb = mat_rgb.data();
    d.mat_ior = mat_ior.data();
    mesh_off[1] = (int32_t)(tris.size() / 9);
    d.n_meshes = 1;
    d.mesh_offset = mesh_off.data();
    d.mesh_mat = mesh_mat.data();
    d.mesh_translation = mesh_xlate.data();
    d.n_triangles = (int32_t)(tris.size() / 9);
    d.triangles = tris.data();
    d.n_params = 1;
    d.bindings = bindings.data();
    return d;
  }
};

// Walks the 4-wide tree: every triangle reached exactly once, each leaf box
// holds its triangles' vertices, depth within kMaxDepth4.  Returns the depth.
static int check_tree(const HostScene& hs, int n_tris) {
  std::vector<int> seen(hs.tris.size(), 0);
  int max_depth = 0;
  struct Item { int node, depth; };
  std::vector<Item> todo;
  for (int i = 0; i < PRDPT_MAX_INSTANCES; ++i)
    if (hs.hdr.inst_root[i] >= 0 && i < hs.hdr.n_inst) todo.push_back({hs.hdr.inst_root[i], 1});
  while (!todo.empty()) {
    Item it = todo.back();
    todo.pop_back();
    CHECK(it.node >= 0 && it.node < (int)hs.nodes.size());
    if (it.node < 0 || it.node >= (int)hs.nodes.size()) continue;
    max_depth = std::max(max_depth, it.depth);
    const Node& nd = hs.nodes[it.node];
    for (int c = 0; c < 4; ++c) {
      const int32_t r = nd.ref[c];
      if (r == kEmptyChild) {
        CHECK(nd.lox[c] > nd.hix[c]);  // inverted box: never hit
        continue;
      }
      if (r >= 0) {
        CHECK(r > it.node);  // depth-first layout: a subtree follows its node
        todo.push_back({r, it.depth + 1});
        continue;
      }
      const int code = ~r, first = code >> 3, count = (code & 7) + 1;
      CHECK(count <= kLeafMax);
      CHECK(first >= 0 && first + count <= (int)hs.tris.size());
      for (int t = first; t < first + count && t < (int)hs.tris.size(); ++t) {
        seen[t]++;
        const Tri& tr = hs.tris[t];
        const float v[3][3] = {{tr.v0x, tr.v0y, tr.v0z},
                               {tr.v0x + tr.e1x, tr.v0y + tr.e1y, tr.v0z + tr.e1z},
                               {tr.v0x + tr.e2x, tr.v0y + tr.e2y, tr.v0z + tr.e2z}};
        for (int k = 0; k < 3; ++k) {
          CHECK(nd.lox[c] <= v[k][0] && v[k][0] <= nd.hix[c]);
          CHECK(nd.loy[c] <= v[k][1] && v[k][1] <= nd.hiy[c]);
          CHECK(nd.loz[c] <= v[k][2] && v[k][2] <= nd.hiz[c]);
        }
      }
    }
  }
  CHECK((int)hs.tris.size() == n_tris);
  for (size_t t = 0; t < seen.size(); ++t) CHECK(seen[t] == 1);
  CHECK(max_depth <= kMaxDepth4);
  return max_depth;
}

static void random_soup(SceneArrays& a, int n, float extent, float size, unsigned seed) {
  std::mt19937 rng(seed);
  std::uniform_real_distribution<float> u(-1.0f, 1.0f);
  a.tris.clear();
  for (int i = 0; i < n; ++i) {
    const float c[3] = {u(rng) * extent, u(rng) * extent, u(rng) * extent};
    for (int k = 0; k < 3; ++k)
      for (int ax = 0; ax < 3; ++ax) a.tris.push_back(c[ax] + u(rng) * size);
  }
}

// One lane of the render kernel's node loop, replayed on the host to check the
// traversal stack bound.  Every box the ray meets is kept (no distance
// culling: the most entries), and the decisions the other lanes of a wave
// make are drawn at random: whether a visit takes the branch-free placement
// (only possible while this lane is four entries or more from the LDS part's
// end) or the branchy one, when the wave turns to the leaf phase (which
// clears the pending leaf), and when it suspends the query (the node being
// visited goes back on the stack).  The placement and pop rules are the
// kernel's: the nearest hit child visited next when inner, else made the
// pending leaf or pushed on top; a lane holding a leaf pops inner entries
// only.  Returns the deepest stack; *overflow is set when a push would pass
// kStackBound.
static int emulate_lane(const HostScene& hs, const float o[3], const float d[3], std::mt19937& rng,
                        bool* overflow) {
  const float inf = INFINITY;
  float inv[3], oi[3];
  for (int a = 0; a < 3; ++a) {
    const float x = std::fabs(d[a]) < 1e-20f ? std::copysign(1e-20f, d[a]) : d[a];
    inv[a] = 1.0f / x;
    oi[a] = -o[a] * inv[a];
  }
  std::vector<int> st(kStackBound + 4, 0);
  int sp = 0, node = -1, leaf = 0, deepest = 0;
  auto push = [&](int e) {
    if (sp >= kStackBound) {
      *overflow = true;
      return;
    }
    st[sp++] = e;
    deepest = std::max(deepest, sp);
  };
  push(hs.hdr.inst_root[0]);
  for (long long it = 0; it < 50000000LL; ++it) {
    const int e = sp > 0 ? st[sp - 1] : 0;
    if (node < 0 && sp > 0 && (leaf == 0 || e >= 0)) {
      --sp;
      if (e < 0) leaf = e;
      else node = e;
    }
    if (node < 0 && leaf == 0 && sp == 0) break;
    const bool ready = leaf != 0 || (node < 0 && sp == 0);
    if (rng() % (ready ? 3 : 5) == 0) {  // the wave breaks (all ready, or the leaf quorum)
      leaf = 0;  // the leaf phase
      if (node >= 0 && rng() % 6 == 0) {  // suspended: resumes with an empty hand
        push(node);
        node = -1;
      }
      continue;
    }
    if (node < 0) continue;
    const Node& nd = hs.nodes[node];
    float t[4];
    int r[4];
    for (int c = 0; c < 4; ++c) {
      const float lo[3] = {nd.lox[c], nd.loy[c], nd.loz[c]}, hi[3] = {nd.hix[c], nd.hiy[c], nd.hiz[c]};
      float tmin = 0.0f, tmax = inf;
      for (int a = 0; a < 3; ++a) {
        const float t0 = lo[a] * inv[a] + oi[a], t1 = hi[a] * inv[a] + oi[a];
        tmin = std::max(tmin, std::min(t0, t1));
        tmax = std::min(tmax, std::max(t0, t1));
      }
      t[c] = (lo[0] <= hi[0] && tmin <= tmax) ? tmin : inf;
      r[c] = nd.ref[c];
    }
    auto order2 = [&](int a, int b) {
      if (t[b] < t[a]) {
        std::swap(t[a], t[b]);
        std::swap(r[a], r[b]);
      }
    };
    order2(0, 1);
    order2(2, 3);
    order2(0, 2);
    order2(1, 3);
    order2(1, 2);
    node = -1;
    if (sp <= kStackEntries - 4 && rng() % 4 != 0) {  // branch-free placement
      const int h = (t[0] < inf) + (t[1] < inf) + (t[2] < inf) + (t[3] < inf);
      for (int i = h - 1; i >= 1; --i) push(r[i]);
      if (h > 0) {
        if (r[0] >= 0) node = r[0];
        else if (leaf == 0) leaf = r[0];
        else push(r[0]);
      }
    } else {  // branchy placement: nearest inner child next, nearest leaf pending
      int next = -1, near_leaf = 0;
      for (int i = 3; i >= 0; --i) {
        if (!(t[i] < inf)) continue;
        if (r[i] >= 0) {
          if (next >= 0) push(next);
          next = r[i];
        } else {
          if (near_leaf != 0) push(near_leaf);
          near_leaf = r[i];
        }
      }
      if (near_leaf != 0) {
        if (leaf == 0) leaf = near_leaf;
        else push(near_leaf);
      }
      node = next;
    }
  }
  return deepest;
}

// Deepest emulated stack over `rays` rays aimed from around the tree's bounds
// at points inside them.
static int emulate_rays(const HostScene& hs, int rays, unsigned seed) {
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  const Node& root = hs.nodes[hs.hdr.inst_root[0]];
  for (int c = 0; c < 4; ++c) {
    if (root.ref[c] == kEmptyChild) continue;
    const float l[3] = {root.lox[c], root.loy[c], root.loz[c]}, h[3] = {root.hix[c], root.hiy[c], root.hiz[c]};
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], l[a]);
      hi[a] = std::max(hi[a], h[a]);
    }
  }
  std::mt19937 rng(seed);
  std::uniform_real_distribution<float> u(0.0f, 1.0f);
  int deepest = 0;
  bool overflow = false;
  for (int i = 0; i < rays; ++i) {
    float o[3], d[3], len = 0.0f;
    for (int a = 0; a < 3; ++a) {
      const float ext = hi[a] - lo[a];
      o[a] = lo[a] - 0.5f * ext + 2.0f * ext * u(rng);
      d[a] = lo[a] + ext * u(rng) - o[a];
      len += d[a] * d[a];
    }
    if (!(len > 0.0f)) continue;
    for (int a = 0; a < 3; ++a) d[a] /= std::sqrt(len);
    deepest = std::max(deepest, emulate_lane(hs, o, d, rng, &overflow));
  }
  CHECK(!overflow);
  CHECK(deepest <= kStackBound);
  return deepest;
}

int main(int argc, char** argv) {
  // ---- the GPU tests' deep-stack scene (raw float32 [n][9] triangles): its
  // tree must stay within the stack bound while exceeding the LDS part
  if (argc > 1) {
    FILE* f = std::fopen(argv[1], "rb");
    CHECK(f != nullptr);
    if (f) {
      SceneArrays a;
      float buf[9];
      while (std::fread(buf, sizeof(float), 9, f) == 9) a.tris.insert(a.tris.end(), buf, buf + 9);
      std::fclose(f);
      prdpt_scene_desc d = a.desc();
      HostScene hs;
      CHECK(build_host_scene(&d, hs) == PRDPT_OK);
      const int depth = check_tree(hs, (int)(a.tris.size() / 9));
      std::printf("file depth4=%d stack_bound=%d lds_entries=%d\n", depth, 3 * depth + 1,
                  kStackEntries);
      std::printf("file emulated deepest stack=%d\n", emulate_rays(hs, 24, 5u));
    }
  }
  // ---- BVH builds and invariants
  const int sizes[] = {1, 2, 3, 4, 5, 17, 33, 1000, 20000};
  for (int n : sizes) {
    SceneArrays a;
    random_soup(a, n, 1.0f, 0.05f, 100u + n);
    prdpt_scene_desc d = a.desc();
    HostScene hs;
    CHECK(build_host_scene(&d, hs) == PRDPT_OK);
    const int depth = check_tree(hs, n);
    std::printf("soup n=%d nodes=%zu depth4=%d emulated deepest stack=%d\n", n, hs.nodes.size(),
                depth, emulate_rays(hs, n >= 1000 ? 64 : 16, 17u + n));
  }
  {  // every triangle identical: no split separates them
    SceneArrays a;
    for (int i = 0; i < 300; ++i)
      for (float v : {0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f, 0.f}) a.tris.push_back(v);
    prdpt_scene_desc d = a.desc();
    HostScene hs;
    CHECK(build_host_scene(&d, hs) == PRDPT_OK);
    std::printf("identical depth4=%d\n", check_tree(hs, 300));
  }
  {  // zero-area and huge triangles
    SceneArrays a;
    random_soup(a, 500, 1e6f, 0.0f, 7u);
    prdpt_scene_desc d = a.desc();
    HostScene hs;
    CHECK(build_host_scene(&d, hs) == PRDPT_OK);
    std::printf("degenerate depth4=%d\n", check_tree(hs, 500));
  }
  {  // a deep tree of long, thin, overlapping triangles across the view: a
     // ray meets most boxes, so traversal keeps up to three siblings per level
    SceneArrays a;
    std::mt19937 rng(3);
    std::uniform_real_distribution<float> u(-1.0f, 1.0f);
    const int n = 65536;
    for (int i = 0; i < n; ++i) {
      const float z = u(rng) * 0.5f, x = u(rng), y = u(rng), dx = u(rng), dy = u(rng);
      const float tri[9] = {x - dx, y - dy, z, x + dx, y + dy, z + 0.001f, x + 0.002f, y, z};
      for (float v : tri) a.tris.push_back(v);
    }
    prdpt_scene_desc d = a.desc();
    HostScene hs;
    CHECK(build_host_scene(&d, hs) == PRDPT_OK);
    const int depth = check_tree(hs, n);
    std::printf("deep depth4=%d stack_bound=%d lds_entries=%d private_entries=%d\n", depth,
                3 * depth + 1, kStackEntries, kStackOverflow);
    std::printf("deep emulated deepest stack=%d\n", emulate_rays(hs, 64, 9u));
    CHECK(3 * depth + 1 <= kStackBound);
  }
  // ---- the division-free quad coordinate test decides as the division does:
  // (x <= lo || x > nn) == (round(x / nn) < 0 || round(x / nn) > 1)
  {
    std::mt19937 rng(11);
    std::uniform_real_distribution<float> ue(-140.0f, 120.0f);
    long long checked = 0, mismatches = 0;
    auto agree = [&](float x, float nn, float lo) {
      const float q = x / nn;
      const bool div = q < 0.0f || q > 1.0f;
      const bool cmp = x <= lo || x > nn;
      ++checked;
      if (div != cmp) ++mismatches;
    };
    auto step = [](float v, int k) {
      while (k > 0) { v = std::nextafter(v, INFINITY); --k; }
      while (k < 0) { v = std::nextafter(v, -INFINITY); ++k; }
      return v;
    };
    std::vector<float> nns = {1.0f, 2.0f, 1.5f, 3.99f, 160000.0f, 3.0e38f, 1e-30f, 1.2e-38f,
                              0.0625f, 1.0000001f, 1.9999999f};
    for (int i = 0; i < 3000; ++i) nns.push_back(std::ldexp(1.0f + (float)(rng() % 1000) / 1000.0f,
                                                            (int)ue(rng)));
    for (float nn : nns) {
      if (!(nn > 0.0f) || !std::isfinite(nn)) continue;
      const float lo = quad_neg_limit_host(nn);
      for (float c : {0.0f, -0.0f, lo, nn, -nn, std::ldexp(nn, -150), -std::ldexp(nn, -150),
                      1.0f, -1.0f})
        for (int k = -40; k <= 40; ++k) agree(step(c, k), nn, lo);
      for (int k = 0; k < 200; ++k) {
        uint32_t b = (uint32_t)rng();
        float x;
        std::memcpy(&x, &b, 4);
        agree(x, nn, lo);
      }
    }
    std::printf("quad limits: %lld cases, %lld mismatches\n", checked, mismatches);
    CHECK(mismatches == 0);
  }
  // ---- validation failures
  {
    SceneArrays a;
    random_soup(a, 10, 1.0f, 0.1f, 9u);
    prdpt_scene_desc d = a.desc();
    HostScene hs;
    prdpt_scene_desc bad = d;
    bad.width = 0;
    CHECK(build_host_scene(&bad, hs) == PRDPT_E_SCENE);
    bad = d;
    bad.n_params = 0;
    CHECK(build_host_scene(&bad, hs) == PRDPT_E_SCENE);
    bad = d;
    bad.triangles = nullptr;
    CHECK(build_host_scene(&bad, hs) == PRDPT_E_SCENE);
    std::vector<int32_t> bad_bind{2, 5, 0};  // mesh index out of range
    bad = d;
    bad.bindings = bad_bind.data();
    CHECK(build_host_scene(&bad, hs) == PRDPT_E_SCENE);
    std::vector<int32_t> bad_mat{7};
    bad = d;
    bad.mesh_mat = bad_mat.data();
    CHECK(build_host_scene(&bad, hs) == PRDPT_E_SCENE);
    CHECK(build_host_scene(nullptr, hs) == PRDPT_E_ARG);
  }
  // ---- entry points reject null arguments before touching a device
  CHECK(prdpt_ctx_create(0, nullptr, 0, nullptr) == PRDPT_E_ARG);
  CHECK(prdpt_ctx_destroy(nullptr) == PRDPT_E_ARG);
  CHECK(prdpt_scene_create(nullptr, nullptr, nullptr, nullptr) == PRDPT_E_ARG);
  CHECK(prdpt_scene_destroy(nullptr) == PRDPT_E_ARG);
  CHECK(prdpt_grad_estimate(nullptr, nullptr, nullptr, nullptr, 4, 1, 0, nullptr, nullptr,
                            nullptr) == PRDPT_E_ARG);
  CHECK(prdpt_grad_estimate_async(nullptr, nullptr, nullptr, nullptr, 4, 1, 0, nullptr, nullptr,
                                  nullptr, nullptr) == PRDPT_E_ARG);
  CHECK(prdpt_combine_async(nullptr, 1, 1, nullptr, nullptr, nullptr, nullptr, 0) == PRDPT_E_ARG);
  CHECK(prdpt_batch_estimate(nullptr, nullptr, 0) == PRDPT_E_ARG);
  CHECK(prdpt_server_start(nullptr, nullptr, nullptr) == PRDPT_E_ARG);
  CHECK(prdpt_server_submit_deadline(nullptr, 0, nullptr, nullptr, 4, 1, 0, 1.0, nullptr) ==
        PRDPT_E_ARG);
  CHECK(prdpt_debug_fail_allocations(-1) == PRDPT_OK);
  // ---- host optimiser step
  {
    double theta[3] = {1.0, -2.0, 0.5}, g[3] = {0.1, -0.2, 0.0}, m[3] = {0, 0, 0}, v[3] = {0, 0, 0};
    CHECK(prdpt_adam_step(3, theta, g, m, v, 1, 0.01, 0.9, 0.999, 1e-8) == PRDPT_OK);
    CHECK(std::fabs(theta[0] - (1.0 - 0.01)) < 1e-9 && std::fabs(theta[1] - (-2.0 + 0.01)) < 1e-9);
    CHECK(prdpt_adam_step(3, nullptr, g, m, v, 1, 0.01, 0.9, 0.999, 1e-8) == PRDPT_E_ARG);
    CHECK(prdpt_sigma_schedule(1.0, 0.05, 0, 200) == 1.0);
    CHECK(std::fabs(prdpt_sigma_schedule(1.0, 0.05, 199, 200) - 0.05) < 1e-15);
  }
  // ---- a context on a missing device fails cleanly
  {
    prdpt_ctx* ctx = nullptr;
    const int rc = prdpt_ctx_create(999, nullptr, 0, &ctx);
    CHECK(rc != PRDPT_OK && ctx == nullptr);
  }
  if (g_failures) {
    std::fprintf(stderr, "%d checks failed\n", g_failures);
    return 1;
  }
  std::printf("host checks OK\n");
  return 0;
}
