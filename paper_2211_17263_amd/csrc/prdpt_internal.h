// Internal layouts shared by the host API (api.cpp, bvh.cpp) and the kernels.
#pragma once
#include <stdint.h>

#include "prdpt.h"

namespace prdpt {

constexpr int kTagTau = 1;
constexpr int kTagPath = 2;
constexpr int kTagRef = 3;
constexpr int kMaxInnerDepth = 25;               // BVH inner-node depth bound (root = 1)
// Traversal stack entries per ray: each inner node on the current path keeps at
// most one child on the stack, and the last one visited at most two (both
// children leaves while a leaf is already pending), so depth + 1 suffice.
constexpr int kStackEntries = kMaxInnerDepth + 1;

// Flattened BVH node: both children's boxes live in the parent (64 bytes, four
// 16-byte loads).  cnt == 0: idx is an inner node; cnt > 0: idx is the first of
// cnt triangles.  Boxes are padded outward so the binary32 slab test is
// conservative for every binary32 triangle hit inside them.
struct alignas(16) Node {
  float c0lox, c0hix, c0loy, c0hiy;
  float c1lox, c1hix, c1loy, c1hiy;
  float c0loz, c0hiz, c1loz, c1hiz;
  int32_t idx0, idx1, cnt0, cnt1;
};
static_assert(sizeof(Node) == 64, "node layout");

// Triangle: v0, e1 = v1 - v0, e2 = v2 - v0 (binary32, computed on the host),
// global primitive id and material (48 bytes, three 16-byte loads).
struct alignas(16) Tri {
  float v0x, v0y, v0z, e1x;
  float e1y, e1z, e2x, e2y;
  float e2z;
  int32_t id, mat, pad;
};
static_assert(sizeof(Tri) == 48, "triangle layout");

// Small per-scene constants; each work-group copies this to LDS and applies its
// perturbation's parameter values.
struct SceneHdr {
  float eye[3], fwd[3], right[3], up[3], env[3];
  int32_t W, H, spp, B, pixel_center;
  int32_t n_mat, n_sph, n_quad, n_inst, n_pl, n_param, n_area, n_tri;
  int32_t tri_id_base;                       // n_sph + n_quad
  int32_t mat_type[PRDPT_MAX_MATERIALS];
  float mat_rgb[PRDPT_MAX_MATERIALS][3];
  float mat_ior[PRDPT_MAX_MATERIALS];
  float sph[PRDPT_MAX_SPHERES][4];
  int32_t sph_mat[PRDPT_MAX_SPHERES];
  float quad[PRDPT_MAX_QUADS][9];
  int32_t quad_mat[PRDPT_MAX_QUADS];
  int32_t area_quad[PRDPT_MAX_QUADS];        // emissive quads in index order
  int32_t inst_root[PRDPT_MAX_INSTANCES];    // root node of each instance BVH (-1: empty)
  float inst_xlate[PRDPT_MAX_INSTANCES][3];
  float pl[PRDPT_MAX_POINT_LIGHTS][6];
  int32_t bind_kind[PRDPT_MAX_PARAMS];
  int32_t bind_index[PRDPT_MAX_PARAMS];      // instance index for meshes
  int32_t bind_comp[PRDPT_MAX_PARAMS];
};

// Device-side view of a resident scene.
struct DevScene {
  const SceneHdr* hdr;
  const Node* nodes;
  const Tri* tris;
};

// One request of a batch (device table, filled by the host per batch).  Rows
// of X/tau/c use the fixed stride PRDPT_MAX_PARAMS.
struct BatchReq {
  DevScene scene;
  const float* ref;
  int32_t W, H, N, d, n_tiles, items_per_row, est, pad0;
  uint32_t k0, k1;
  int32_t item_base, pair_base, row_base, partial_base;
  double cd, sqrt2pi, inv_den;
  float theta[PRDPT_MAX_PARAMS];
  float sigma[PRDPT_MAX_PARAMS];
};

// Batch totals and the work counter of the persistent render kernel.
struct BatchMeta {
  int32_t n_req, total_pairs, total_items, total_rows;
  int32_t tiles_per_item, counter, pad0, pad1;
};

// Host-side BVH build result for one instance.
struct BvhOut {
  int root;          // index into the global node array
  int depth;
};

}  // namespace prdpt
