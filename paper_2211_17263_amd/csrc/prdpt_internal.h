// Internal layouts shared by the host API (api.cpp, bvh.cpp) and the kernels.
#pragma once
#include <stdint.h>

#include "prdpt.h"

namespace prdpt {

constexpr int kTagTau = 1;
constexpr int kTagPath = 2;
constexpr int kTagRef = 3;
constexpr int kMaxInnerDepth = 25;  // depth bound of the binary tree the builder makes (root = 1)
// The device BVH is 4-wide: each node opens two levels of the binary tree, so
// its depth is at most (kMaxInnerDepth + 1) / 2.
constexpr int kMaxDepth4 = (kMaxInnerDepth + 1) / 2;
// Traversal stack entries per ray: every node on the current path keeps at
// most three of its children on the stack and the last one visited at most
// four (its nearest child a leaf while a leaf is already pending: that leaf
// goes on top, and a lane holding a leaf pops no leaf, so the lane descends
// no further until the leaf phase); a suspended node adds one entry for
// itself.  kStackEntries live in LDS, the rest in a
// small per-lane private array that only unusually deep descents reach.
constexpr int kStackBound = 3 * kMaxDepth4 + 1;
// 13 LDS entries keep a render work-group (with one sphere) within 7680
// bytes of LDS: gfx950 hands out a CU's 160 KB of LDS in units of 1280 bytes
// (measured: 21 work-groups of 7680 bytes are resident on a CU at once, 18
// of 7696 to 8960 bytes), so 20 work-groups, five waves per SIMD, fit; deeper
// entries (a descent past 13 pending entries) go to the private part.
#ifndef PRDPT_STACK_LDS
#define PRDPT_STACK_LDS 13
#endif
// LDS allocation unit of a work-group on gfx950 (bytes)
constexpr int kLdsAllocUnit = 1280;
constexpr int kStackEntries = PRDPT_STACK_LDS;
constexpr int kStackOverflow = kStackBound - kStackEntries;
// child reference of an empty slot of a 4-wide node
constexpr int32_t kEmptyChild = INT32_MIN;
// most triangles in a BVH leaf (the traversal spreads a wave's pending leaves
// over its lanes in a table of kLeafMax entries per lane)
#ifndef PRDPT_LEAF_MAX
#define PRDPT_LEAF_MAX 4
#endif
constexpr int kLeafMax = PRDPT_LEAF_MAX;

// Flattened 4-wide BVH node (128 bytes, seven 16-byte loads): the padded boxes
// of its children as six 4-vectors (one per box face coordinate) and the child
// references.  A reference >= 0 is an inner node, < 0 a leaf of triangles
// encoded as ~(first << 3 | (count - 1)), kEmptyChild an unused slot (whose box
// is inverted, lo = +inf and hi = -inf, so that no ray hits it).  Boxes are
// padded outward so the binary32 slab test is conservative for every binary32
// triangle hit inside them.  Each axis keeps lo and hi 16 bytes apart, which
// lets the traversal load a ray's near and far planes directly.
struct alignas(16) Node {
  float lox[4], hix[4], loy[4], hiy[4], loz[4], hiz[4];
  int32_t ref[4];
  int32_t pad[4];
};
static_assert(sizeof(Node) == 128, "node layout");

// Triangle: v0, e1 = v1 - v0, e2 = v2 - v0 (binary32, computed on the host),
// global primitive id, material and instance (48 bytes, three 16-byte loads).
struct alignas(16) Tri {
  float v0x, v0y, v0z, e1x;
  float e1y, e1z, e2x, e2y;
  float e2z;
  int32_t id, mat, inst;  // instance index (its rotation turns the normal into the world)
};
static_assert(sizeof(Tri) == 48, "triangle layout");

// Small per-scene constants; each work-group copies this part to LDS and
// applies its perturbation's parameter values.
struct SceneLds {
  float eye[3], fwd[3], right[3], up[3], env[3];
  int32_t W, H, spp, B, pixel_center;
  int32_t n_mat, n_sph, n_quad, n_inst, n_pl, n_param, n_area, n_tri;
  int32_t tri_id_base;                       // n_sph + n_quad
  float inv_w, inv_h;                        // 1/W, 1/H when W, H are powers of two, else 0
  int32_t tile_log2;                         // render tiles of 2^tile_log2 square pixels (3 or 2)
  int32_t mat_type[PRDPT_MAX_MATERIALS];
  float mat_rgb[PRDPT_MAX_MATERIALS][3];     // a dielectric's [0] holds 1/ior (rounded)
  float mat_ior[PRDPT_MAX_MATERIALS];
  float quad[PRDPT_MAX_QUADS][9];
  int32_t quad_mat[PRDPT_MAX_QUADS];
  int32_t area_quad[PRDPT_MAX_QUADS];        // emissive quads in index order
  float quad_n[PRDPT_MAX_QUADS][4];          // edge1 x edge2 and its squared length nn
  float quad_lo[PRDPT_MAX_QUADS];            // largest x whose rounded x / nn is below 0
  float quad_nu[PRDPT_MAX_QUADS][4];         // unit normal and area (edges are never bound)
  int32_t inst_root[PRDPT_MAX_INSTANCES];    // root node of each instance BVH (-1: empty)
  float inst_xlate[PRDPT_MAX_INSTANCES][3];
  float inst_ang[PRDPT_MAX_INSTANCES][3];    // rotation angles (a, b, c)
  float inst_rot[PRDPT_MAX_INSTANCES][9];    // Rz(c) Ry(b) Rx(a), row-major
  int32_t has_rot;                           // some instance is rotated or has a bound angle
  float pl[PRDPT_MAX_POINT_LIGHTS][6];
};

// The whole scene header in device memory: the LDS part, then the spheres
// (copied to a dynamically sized LDS array of n_sph entries, so that scenes
// with few spheres keep the LDS of many resident work-groups) and the
// parameter bindings (read from device memory when a perturbation is applied).
struct SceneHdr : SceneLds {
  float sph[PRDPT_MAX_SPHERES][4];
  int32_t sph_mat[PRDPT_MAX_SPHERES];
  int32_t bind_kind[PRDPT_MAX_PARAMS];
  int32_t bind_index[PRDPT_MAX_PARAMS];      // instance index for meshes
  int32_t bind_comp[PRDPT_MAX_PARAMS];
};

// Dynamic LDS of a render work-group: n_sph spheres (centre, radius) and their
// materials.
inline int sphere_lds_bytes(int n_sph) { return n_sph * (4 * 4 + 4); }

// Device-side view of a resident scene.
struct DevScene {
  const SceneHdr* hdr;
  const Node* nodes;
  const Tri* tris;
  const int32_t* tri_slot;  // index in tris of the triangle with id tri_id_base + i, by i
};

// One request of a batch (device table, filled by the host per batch).  Rows
// of X/tau/c use the fixed stride PRDPT_BATCH_MAX_PARAMS.
struct BatchReq {
  DevScene scene;
  const float* ref;
  int32_t W, H, N, d, n_tiles, items_per_row, est, pad0;
  uint32_t k0, k1;
  int32_t item_base, pair_base, row_base, partial_base;
  double cd, sqrt2pi, inv_den;
  float theta[PRDPT_BATCH_MAX_PARAMS];
  float sigma[PRDPT_BATCH_MAX_PARAMS];
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
