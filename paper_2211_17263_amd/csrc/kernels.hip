// HIP kernels for gfx950 (CDNA4): perturbation prologue, fused path-trace +
// per-image loss, and the binary64 finalisation / gradient combination.
//
// Numerical contract with the CPU reference: everything that decides which
// primitive a ray hits (camera rays, intersection tests, hit points, normals,
// spawn offsets, sampled directions, light sample points, Fresnel choice) is
// evaluated in binary32 in a fixed order without contraction (the library is
// built with -ffp-contract=off and correctly rounded division and square root),
// and the sample transforms use the library's own ln / sincos(2 pi u) built from
// basic IEEE operations.  Signed zeros count too: the sign of a zero normal
// component picks the tangent frame of a bounce, so a triangle's world normal
// is always the instance rotation applied to its mesh-frame normal, even where
// that rotation is the identity.  Per-sample paths are therefore reproducible
// bit for bit on any IEEE-754 machine; only the pixel/loss sums differ in
// rounding.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "exact_math.h"
#include "prdpt_internal.h"

namespace prdpt {
namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and sample transforms
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32->64 product gives both halves
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// (0,1) uniform from the top 23 bits: ((x >> 9) + 1/2) 2^-23, exact in binary32
__device__ __forceinline__ float unit_open(uint32_t x) {
  return ((float)(x >> 9) + 0.5f) * 1.1920928955078125e-07f;
}

// ln for positive normal input: reduce to m in [sqrt(1/2), sqrt(2)], then
// ln m = 2 atanh((m-1)/(m+1)) by the odd series through s^11, plus e ln 2 in two parts
__device__ __forceinline__ float log_ieee(float x) {
  uint32_t b = __float_as_uint(x);
  int e = (int)((b >> 23) & 0xffu) - 127;
  float m = __uint_as_float((b & 0x007fffffu) | 0x3f800000u);
  if (m > 1.41421356f) {
    m = m * 0.5f;
    e = e + 1;
  }
  const float s = (m - 1.0f) / (m + 1.0f);
  const float s2 = s * s;
  float p = 1.0f / 11.0f;
  p = 1.0f / 9.0f + s2 * p;
  p = 1.0f / 7.0f + s2 * p;
  p = 1.0f / 5.0f + s2 * p;
  p = 1.0f / 3.0f + s2 * p;
  const float at = s + s * (s2 * p);
  const float lm = at + at;
  const float fe = (float)e;
  return fe * 0.693145751953125f + (lm + fe * 1.42860677e-06f);
}

// sin and cos of 2 pi u, u in [0,1): quarter-turn index plus remainder in
// [-1/8, 1/8] (exact), Taylor series of sin through x^9 and cos through x^10
__device__ __forceinline__ void sincos_turn(float u, float* so, float* co) {
  const float u4 = u * 4.0f;
  int q = (int)u4;
  float r = u - (float)q * 0.25f;
  if (r > 0.125f) {
    r = r - 0.25f;
    q = q + 1;
  }
  const float x = r * 6.28318530717958647692f;
  const float x2 = x * x;
  float ps = -1.0f / 5040.0f + x2 * (1.0f / 362880.0f);
  ps = 1.0f / 120.0f + x2 * ps;
  ps = -1.0f / 6.0f + x2 * ps;
  const float sn = x + x * (x2 * ps);
  float pc = 1.0f / 40320.0f + x2 * (-1.0f / 3628800.0f);
  pc = -1.0f / 720.0f + x2 * pc;
  pc = 1.0f / 24.0f + x2 * pc;
  pc = -0.5f + x2 * pc;
  const float cs = 1.0f + x2 * pc;
  switch (q & 3) {
    case 0: *so = sn; *co = cs; break;
    case 1: *so = cs; *co = -sn; break;
    case 2: *so = -sn; *co = -cs; break;
    default: *so = -cs; *co = sn; break;
  }
}

// ---------------------------------------------------------------------------
// binary32 vector helpers with a fixed evaluation order
// ---------------------------------------------------------------------------
struct V3 {
  float x, y, z;
};
__device__ __forceinline__ V3 mk(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 sub(V3 a, V3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 neg(V3 a) { return mk(-a.x, -a.y, -a.z); }
__device__ __forceinline__ V3 scale(V3 a, float s) { return mk(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
// a / |a|: the correctly rounded root of the squared length, its correctly
// rounded reciprocal (the root of a non-negative float is +0, a normal number
// below 2^64, +inf or NaN: recip_nr's domain) and three products
__device__ __forceinline__ V3 unit(V3 a) {
  const float len = sqrt_cr(dot(a, a));
  const float inv = recip_nr(len);
  return scale(a, inv);
}
__device__ __forceinline__ V3 at(V3 o, V3 d, float t) {
  return mk(o.x + d.x * t, o.y + d.y * t, o.z + d.z * t);
}
__device__ __forceinline__ V3 ld3(const float* p) { return mk(p[0], p[1], p[2]); }

// ---------------------------------------------------------------------------
// primitive tests: accept t in (0, tmax)
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool hit_sphere(V3 o, V3 d, const float* sp, float tmax, float* tout) {
  const V3 oc = sub(o, ld3(sp));
  const float r = sp[3];
  const float a = dot(d, d);
  const float b = dot(oc, d);
  const float cc = dot(oc, oc) - r * r;
  const float disc = b * b - a * cc;
  if (disc < 0.0f) return false;
  const float sq = sqrt_cr(disc);
  const float q = (b >= 0.0f) ? -(b + sq) : -(b - sq);
  if (q == 0.0f) return false;
  const float t0 = q / a, t1 = cc / q;
  const float tn = t0 < t1 ? t0 : t1;
  const float tf = t0 < t1 ? t1 : t0;
  const float t = tn > 0.0f ? tn : tf;
  if (!(t > 0.0f && t < tmax)) return false;
  *tout = t;
  return true;
}

// qn: the quad's edge1 x edge2 and its squared length nn; qlo: the largest x
// whose correctly rounded quotient x / nn is below 0 (per-scene constants).
// A parallelogram coordinate is a numerator X over nn, and the hit needs its
// rounded quotient in [0, 1]; rounding is monotone, 1 is representable and
// nn (1 + 2^-24) lies below the float after nn, so round(X / nn) > 1 exactly
// when X > nn, and round(X / nn) < 0 exactly when X <= qlo: the two tests
// decide as the divisions would, without dividing.
__device__ __forceinline__ bool hit_quad(V3 o, V3 d, const float* qd, const float* qn, float qlo,
                                         float tmax, float* tout) {
  const V3 qo = ld3(qd), e1 = ld3(qd + 3), e2 = ld3(qd + 6);
  const V3 n = ld3(qn);
  const float den = dot(n, d);
  if (den == 0.0f) return false;
  const float t = dot(n, sub(qo, o)) / den;
  if (!(t > 0.0f && t < tmax)) return false;
  const V3 pd = sub(at(o, d, t), qo);
  const float nn = qn[3];
  const float al = dot(cross(pd, e2), n);
  if (al <= qlo || al > nn) return false;
  const float be = dot(cross(e1, pd), n);
  if (be <= qlo || be > nn) return false;
  *tout = t;
  return true;
}

// Moeller-Trumbore on the stored (v0, e1, e2).  Every quantity is computed
// before any decision so that the three triangle loads are consumed together;
// the accept predicate (det != 0, 0 <= u <= 1, v >= 0, u + v <= 1,
// 0 < t < tmax, each on the rounded binary32 values) is the one a test with
// early returns takes.
__device__ __forceinline__ bool hit_tri(V3 o, V3 d, V3 v0, V3 e1, V3 e2, float tmax, float* tout) {
  const V3 pv = cross(d, e2);
  const float det = dot(e1, pv);
  const V3 tv = sub(o, v0);
  const V3 qv = cross(tv, e1);
  const float un = dot(tv, pv);
  const float vn = dot(d, qv);
  const float tn = dot(e2, qv);
  const float inv = 1.0f / det;
  const float u = un * inv;
  const float v = vn * inv;
  const float t = tn * inv;
  const bool hit = det != 0.0f && !(u < 0.0f || u > 1.0f) && !(v < 0.0f || u + v > 1.0f) &&
                   (t > 0.0f && t < tmax);
  *tout = t;
  return hit;
}

constexpr int kBlock = 64;  // one wave per render tile (8x8 or 4x4 pixels)

struct Hit {
  float t;
  int id;     // global primitive id, -1 = miss
};

__device__ __forceinline__ void keep_closer(Hit& h, float t, int id) {
  if (t < h.t || (t == h.t && id < h.id)) {
    h.t = t;
    h.id = id;
  }
}

// A hit as one 64-bit key whose unsigned order is the (t, primitive id) order
// of keep_closer: t > 0, so its bits order like the value; a miss is
// (inf, all ones), above every hit.
__device__ __forceinline__ unsigned long long hit_key(float t, int id) {
  return ((unsigned long long)__float_as_uint(t) << 32) | (uint32_t)id;
}

// LDS of the leaf phase: the wave's pending (lane, triangle) pairs in lane
// order, as the owning lane of each, and each lane's best hit as a key.  The
// owner table has kLeafMax spare entries: a lane with pairs stores kLeafMax
// entries whatever its count.
struct LeafLds {
  unsigned long long key[kBlock];
  uint8_t owner[kBlock * kLeafMax + kLeafMax];
};
static_assert(kBlock == 64, "the leaf phase spreads pairs over one wave");
static_assert(sizeof(uint8_t) * kBlock * kLeafMax >= sizeof(uint32_t) * kBlock,
              "the deposit claims reuse the leaf phase's owner table");

// LDS of a tile's pixel sums: the radiance of each finished path is added to
// its pixel's entry (tile pixel slot q = x + 8 y).
struct PixLds {
  float rgb[3][kBlock];
};
static_assert(kLeafMax <= 7, "leaf counts are added up from three ballots");
// static LDS of a render work-group: 20 of them (five waves per SIMD) fit a
// CU only within 6 allocation units, with room for one sphere
constexpr size_t kRenderStaticLds = sizeof(SceneLds) + sizeof(int) * kStackEntries * kBlock +
                                    sizeof(float) * (kBlock / 64) + 2 * sizeof(int) +
                                    sizeof(LeafLds) + sizeof(PixLds);
static_assert(kRenderStaticLds + 20 <= 6 * kLdsAllocUnit,
              "the render work-group's LDS must stay within six allocation units");

// Work counters of the instrumented kernel copy: lane-level work (nodes,
// triangles, rays, paths) and wave-level loop iterations (counted once per wave
// by its first active lane), whose ratio is the SIMD efficiency of each loop.
struct Counters {
  uint32_t nodes, tris, rays, paths;
  uint32_t wave_node_iters, wave_tri_iters, wave_outer_iters;
  uint32_t idle_lane_iters;  // ray-loop iterations x lanes with no path of the tile left
  uint32_t overflow_pushes;  // stack pushes into the private part
  uint32_t deepest;          // most stack entries in use at once
};

__device__ __forceinline__ bool first_active_lane() {
  const unsigned long long m = __ballot(1);
  return (int)__lane_id() == __ffsll((long long)m) - 1;
}

// Conservative binary32 slab test of a padded child box, given per axis the
// plane the ray meets first (near) and last (far); returns the entry distance
// (or +inf when the box is missed or lies beyond tcull).  With the planes
// picked by the sign of the inverse direction, fma(near, inv, oi) is the
// smaller of the two plane distances of the axis (the rounded fma is monotone
// in the plane coordinate), so this equals the min/max form of the test.  An
// empty child slot has lo = +inf and hi = -inf on every axis and is missed.
__device__ __forceinline__ float slab(float nx, float fx, float ny, float fy, float nz, float fz,
                                      V3 inv, V3 oi, float tcull) {
  const float tmin = fmaxf(fmaxf(fmaf(nx, inv.x, oi.x), fmaf(ny, inv.y, oi.y)),
                           fmaxf(fmaf(nz, inv.z, oi.z), 0.0f));
  const float tmax = fminf(fminf(fmaf(fx, inv.x, oi.x), fmaf(fy, inv.y, oi.y)),
                           fminf(fmaf(fz, inv.z, oi.z), tcull));
  return tmin <= tmax ? tmin : __builtin_huge_valf();
}

// Byte offset within a node of the four near planes of each axis: lo (x at
// 0, y at 32, z at 64) where the inverse direction is positive, hi (16 bytes
// further) where it is negative; the far planes are at offset ^ 16.
__device__ __forceinline__ uint32_t near_planes(float inv_axis, uint32_t lo_offset) {
  return lo_offset | ((__float_as_uint(inv_axis) >> 27) & 16u);
}

__device__ __forceinline__ float safe_inv(float x) {
  const float ax = fabsf(x) < 1e-20f ? copysignf(1e-20f, x) : x;
  return __builtin_amdgcn_rcpf(ax);
}

// Ray queries over the analytic primitives and every instance BVH.  any =
// true: shadow query, stop at the first occluder with t < tmax (emissive quads
// are not occluders); otherwise keep the closest hit by (t, primitive id), a
// result that does not depend on the order in which primitives are visited.
//
// A query is resumable: begin_trace tests the analytic primitives and queues
// the first instance's root; continue_trace then traverses until the query is
// answered, the wave has spent `budget` node-loop iterations in this call, or
// at least half of the lanes that entered the call have their answer, so
// lanes whose ray is done can shade and start their next ray while long
// traversals go on.  The suspended state is the best hit so far, the stack
// pointer and the instance (Trav); the node being visited is pushed back on the
// lane's stack and the instance-space ray is rebuilt on resumption.
//
// Traversal is "while-while" with postponed leaves: the node loop visits inner
// nodes, and a hit leaf child becomes the lane's pending leaf (or is pushed if
// one is already pending); lanes holding a leaf keep descending speculatively,
// into the nearest inner child and into inner nodes popped from the stack
// (they stop at a leaf on top).  The wave leaves the node loop once every lane
// holds a leaf or has no work left, or once at least PRDPT_LEAF_QUORUM percent
// of its active lanes hold one.  The leaf phase then lists the (lane, triangle) pairs of all pending
// leaves and deals them out to every active lane, a pair per lane per round:
// the lane fetches the owner's ray with cross-lane permutes, tests the
// triangle and folds the hit into the owner's best-hit key in LDS with an
// atomic minimum.  Lanes without a leaf of their own thus test triangles too,
// and a wave spends ceil(pairs / active lanes) rounds instead of the largest
// leaf's count.  Instances are visited in order, each to completion.
//
// Stack entries: >= 0 inner node, < 0 leaf encoded as ~(first << 3 |
// (count - 1)).  The stack holds kStackEntries entries in LDS (stride =
// work-group size) and the rest in the lane's private overflow array; the
// builder bounds the 4-wide depth, every node on the current path keeps at
// most three of its children on the stack and the last visited one at most
// four, and a suspended node adds one entry for itself, so the two parts
// together (kStackBound entries) cannot overflow.
#ifndef PRDPT_LEAF_QUORUM
#define PRDPT_LEAF_QUORUM 25
#endif
#ifndef PRDPT_TRACE_BUDGET
#define PRDPT_TRACE_BUDGET 32
#endif
#ifndef PRDPT_TRACE_QUORUM
#define PRDPT_TRACE_QUORUM 50
#endif

// popcount of the mask's bits below this lane
__device__ __forceinline__ uint32_t mbcnt64(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// the value of x in the lane whose index is addr / 4
__device__ __forceinline__ float bperm(int addr, float x) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(x)));
}

// Per-lane traversal stack: entries [0, kStackEntries) in LDS (stride = the
// work-group size), deeper ones in the lane's private overflow array.
__device__ __forceinline__ void push(int* __restrict__ lds, int stride, int* __restrict__ ovf,
                                     int& sp, int e) {
  if (sp < kStackEntries) {
    lds[sp * stride] = e;
  } else {
    ovf[sp - kStackEntries] = e;
  }
  ++sp;
}

// orders two (distance, reference) pairs by distance
__device__ __forceinline__ void order2(float& ta, int& ra, float& tb, int& rb) {
  const bool sw = tb < ta;
  const float t = sw ? tb : ta;
  const int r = sw ? rb : ra;
  tb = sw ? ta : tb;
  rb = sw ? ra : rb;
  ta = t;
  ra = r;
}

// Rz(c) Ry(b) Rx(a) for the angles (a, b, c) = ang (rotations about the fixed
// x, y, z axes, applied in that order), row-major; entries are formed in
// binary64 and rounded to binary32, so zero angles give the identity exactly,
// and an entry that is zero is +0 (adding +0 clears a negative zero), as in
// the product of the three axis matrices summed from zero.
__host__ __device__ inline void euler_rotation(const float* ang, float* R) {
  const double ca = cos((double)ang[0]), sa = sin((double)ang[0]);
  const double cb = cos((double)ang[1]), sb = sin((double)ang[1]);
  const double cc = cos((double)ang[2]), sc = sin((double)ang[2]);
  R[0] = (float)(cc * cb + 0.0);
  R[1] = (float)(cc * sb * sa - sc * ca + 0.0);
  R[2] = (float)(cc * sb * ca + sc * sa + 0.0);
  R[3] = (float)(sc * cb + 0.0);
  R[4] = (float)(sc * sb * sa + cc * ca + 0.0);
  R[5] = (float)(sc * sb * ca - cc * sa + 0.0);
  R[6] = (float)(-sb + 0.0);
  R[7] = (float)(cb * sa + 0.0);
  R[8] = (float)(cb * ca + 0.0);
}

// The ray (o, d) in the frame of instance `inst`: R^T (o - t) and R^T d
// (without rotations, ROT = false: o - t and d).  R is orthonormal, so the ray
// parameter of a hit is the same in both frames.
template <bool ROT>
__device__ __forceinline__ void to_instance(const SceneLds& S, int inst, V3 o, V3 d, V3& om,
                                            V3& dm) {
  const V3 q = mk(o.x - S.inst_xlate[inst][0], o.y - S.inst_xlate[inst][1],
                  o.z - S.inst_xlate[inst][2]);
  if (ROT) {
    const float* R = S.inst_rot[inst];
    om = mk(R[0] * q.x + R[3] * q.y + R[6] * q.z, R[1] * q.x + R[4] * q.y + R[7] * q.z,
            R[2] * q.x + R[5] * q.y + R[8] * q.z);
    dm = mk(R[0] * d.x + R[3] * d.y + R[6] * d.z, R[1] * d.x + R[4] * d.y + R[7] * d.z,
            R[2] * d.x + R[5] * d.y + R[8] * d.z);
  } else {
    om = q;
    dm = d;
  }
}

struct Trav {
  Hit h;
  int sp;    // stack entries in use
  int inst;  // instance being traversed
};

// first instance at or after i with a BVH, or n_inst
__device__ __forceinline__ int next_inst(const SceneLds& S, int i) {
  while (i < S.n_inst && S.inst_root[i] < 0) ++i;
  return i;
}

// Starts a query: analytic primitives, then the first instance's root on the
// stack.  Returns true when the query is already answered (a shadow ray
// blocked by an analytic primitive, or nothing left to traverse).
template <bool COUNT>
__device__ __forceinline__ bool begin_trace(const SceneLds& S, const float* __restrict__ sph,
                                            V3 o, V3 d, float tmax, bool any, Trav& tr,
                                            int* __restrict__ stack, Counters& cnt) {
  Hit& h = tr.h;
  h.t = __builtin_huge_valf();
  h.id = -1;
  if (COUNT) cnt.rays++;
  for (int i = 0; i < S.n_sph; ++i) {
    float t;
    if (hit_sphere(o, d, sph + 4 * i, tmax, &t)) {
      if (any) {
        h.id = i;
        return true;
      }
      keep_closer(h, t, i);
    }
  }
  for (int i = 0; i < S.n_quad; ++i) {
    if (any && S.mat_type[S.quad_mat[i]] == PRDPT_MAT_EMISSIVE) continue;
    float t;
    if (hit_quad(o, d, S.quad[i], S.quad_n[i], S.quad_lo[i], tmax, &t)) {
      if (any) {
        h.id = S.n_sph + i;
        return true;
      }
      keep_closer(h, t, S.n_sph + i);
    }
  }
  tr.inst = next_inst(S, 0);
  if (tr.inst >= S.n_inst) return true;
  stack[0] = S.inst_root[tr.inst];
  tr.sp = 1;
  return false;
}

// Continues a query; returns true when it is answered (tr.h holds the result).
template <bool COUNT, bool ROT>
__device__ bool continue_trace(const SceneLds& S, const Node* __restrict__ nodes,
                               const Tri* __restrict__ tris, V3 o, V3 d, float tmax, bool any,
                               Trav& tr, int* __restrict__ stack, int stride,
                               int* __restrict__ ovf, LeafLds* __restrict__ lf, int budget,
                               Counters& cnt) {
  Hit& h = tr.h;
  int sp = tr.sp;
  int inst = tr.inst;
  // an instance: the ray in the mesh's own frame
  V3 om, dm;
  to_instance<ROT>(S, inst, o, d, om, dm);
  V3 inv = mk(safe_inv(dm.x), safe_inv(dm.y), safe_inv(dm.z));
  V3 oi = mk(-om.x * inv.x, -om.y * inv.y, -om.z * inv.z);
  int node = -1;   // inner node being visited, -1: none
  int leaf = 0;    // pending leaf (encoded < 0), 0: none
  int iters = 0;
  auto push_entry = [&](int e) {
    push(stack, stride, ovf, sp, e);
    if (COUNT) {
      if (sp > kStackEntries) cnt.overflow_pushes++;
      cnt.deepest = max(cnt.deepest, (uint32_t)sp);
    }
  };
  const int entered = __popcll(__ballot(1));
  while (true) {
    // ---- node loop: descend until enough lanes hold a leaf.  The wave
    // raises its issue priority here: a node visit's loads depend on the
    // previous visit's result, so a wave whose node data has arrived issues
    // ahead of the shading and leaf-phase work of the other waves on the SIMD
    // and has its next loads in flight sooner (the execution of each wave,
    // and so every result, is unchanged)
    __builtin_amdgcn_s_setprio(1);
    while (true) {
      {
        // pop into an empty hand; the LDS read is done by every lane (in
        // bounds) and the private part is read where the top lies beyond the
        // LDS part (in bounds too; the entry is used only where wanted).  A
        // lane holding a pending leaf still pops an inner node from the top
        // (speculative descent), but leaves a leaf entry in place
        const int top = sp - 1;
        int e = stack[max(min(top, kStackEntries - 1), 0) * stride];
        if (__ballot(sp > kStackEntries) != 0ull) {
          if (sp > kStackEntries) e = *(const volatile int*)&ovf[top - kStackEntries];
        }
        const bool want = node < 0 && sp > 0 && (leaf == 0 || e >= 0);
        if (want) {
          sp = top;
          if (e < 0) leaf = e;
          else node = e;
        }
      }
      const bool ready = leaf != 0 || (node < 0 && sp == 0);
      if (__ballot(!ready) == 0ull) break;
#if PRDPT_LEAF_QUORUM < 100
      if (__popcll(__ballot(leaf < 0)) * 100 >= __popcll(__ballot(1)) * PRDPT_LEAF_QUORUM) break;
#endif
      ++iters;
      if (node >= 0) {
        const char* nb = reinterpret_cast<const char*>(nodes);
        const uint32_t at = (uint32_t)node << 7;  // 128-byte nodes
        const uint32_t ax = near_planes(inv.x, at), ay = near_planes(inv.y, at | 32u),
                       az = near_planes(inv.z, at | 64u);
        const float4 nx = *reinterpret_cast<const float4*>(nb + ax);
        const float4 fx = *reinterpret_cast<const float4*>(nb + (ax ^ 16u));
        const float4 ny = *reinterpret_cast<const float4*>(nb + ay);
        const float4 fy = *reinterpret_cast<const float4*>(nb + (ay ^ 16u));
        const float4 nz = *reinterpret_cast<const float4*>(nb + az);
        const float4 fz = *reinterpret_cast<const float4*>(nb + (az ^ 16u));
        const int4 rf = *reinterpret_cast<const int4*>(nb + (at | 96u));
        if (COUNT) {
          cnt.nodes++;
          if (first_active_lane()) cnt.wave_node_iters++;
        }
        const float tcull = any ? tmax : fminf(tmax, h.t);
        const float inf = __builtin_huge_valf();
        float t0 = slab(nx.x, fx.x, ny.x, fy.x, nz.x, fz.x, inv, oi, tcull);
        float t1 = slab(nx.y, fx.y, ny.y, fy.y, nz.y, fz.y, inv, oi, tcull);
        float t2 = slab(nx.z, fx.z, ny.z, fy.z, nz.z, fz.z, inv, oi, tcull);
        float t3 = slab(nx.w, fx.w, ny.w, fy.w, nz.w, fz.w, inv, oi, tcull);
        int r0 = rf.x, r1 = rf.y, r2 = rf.z, r3 = rf.w;  // empty slots: t = inf
        // nearest first (misses last)
        order2(t0, r0, t1, r1);
        order2(t2, r2, t3, r3);
        order2(t0, r0, t2, r2);
        order2(t1, r1, t3, r3);
        order2(t1, r1, t2, r2);
        // far to near: the nearest inner child is visited next and the nearest
        // leaf becomes the pending leaf if none is; the others are pushed so
        // that nearer ones are popped first
        int next = -1, near_leaf = 0;
        if (__ballot(sp > kStackEntries - 4) == 0ull) {
          // a visit pushes at most four entries, and here all of them land in
          // the LDS part.  The h hit children are t0..t(h-1) (misses sort
          // last); children 1..h-1 go on the stack, nearest on top, and the
          // nearest child is visited next when inner, or becomes the pending
          // leaf, or, when a leaf is already pending, goes on top of them
          // (a leaf on top stops the speculative pops until the leaf phase).
          // The stores of kept children are the only branches
          const int h = (int)(t0 < inf) + (int)(t1 < inf) + (int)(t2 < inf) + (int)(t3 < inf);
          const int b = sp + h - 4;  // child i is stored at slot b + 3 - i when i < h
          if (h > 3) stack[b * stride] = r3;
          if (h > 2) stack[(b + 1) * stride] = r2;
          if (h > 1) stack[(b + 2) * stride] = r1;
          sp += max(h - 1, 0);
          // (bitwise operators on the flags keep them lane masks)
          const bool hit0 = h > 0, inner0 = r0 >= 0;
          stack[sp * stride] = r0;  // a free slot, kept only for a second leaf
          sp += (int)(hit0 & !inner0 & (leaf != 0));
          leaf = (hit0 & !inner0 & (leaf == 0)) ? r0 : leaf;
          node = (hit0 & inner0) ? r0 : -1;
          if (COUNT) cnt.deepest = max(cnt.deepest, (uint32_t)sp);
          continue;
        }
        if (t3 < inf) {
          if (r3 >= 0) next = r3;
          else near_leaf = r3;
        }
        if (t2 < inf) {
          if (r2 >= 0) {
            if (next >= 0) push_entry(next);
            next = r2;
          } else {
            if (near_leaf != 0) push_entry(near_leaf);
            near_leaf = r2;
          }
        }
        if (t1 < inf) {
          if (r1 >= 0) {
            if (next >= 0) push_entry(next);
            next = r1;
          } else {
            if (near_leaf != 0) push_entry(near_leaf);
            near_leaf = r1;
          }
        }
        if (t0 < inf) {
          if (r0 >= 0) {
            if (next >= 0) push_entry(next);
            next = r0;
          } else {
            if (near_leaf != 0) push_entry(near_leaf);
            near_leaf = r0;
          }
        }
        if (near_leaf != 0) {
          if (leaf == 0) leaf = near_leaf;
          else push_entry(near_leaf);
        }
        node = next;
      }
    }
    __builtin_amdgcn_s_setprio(0);
    // ---- leaf phase: the pending leaves' (lane, triangle) pairs, spread over
    // the active lanes in lane order; each owner keeps the least hit key of its
    // pairs (the same hit as testing them one by one with keep_closer)
    if (__ballot(leaf != 0) != 0ull) {
      const int lane = (int)__lane_id();
      int n_own = 0, first = 0;
      if (leaf != 0) {
        const int code = ~leaf;
        first = code >> 3;
        n_own = (code & 7) + 1;
        leaf = 0;
      }
      // exclusive prefix sum of the counts over the lanes, and their total
      const unsigned long long c1 = __ballot(n_own & 1), c2 = __ballot(n_own & 2),
                               c4 = __ballot(n_own & 4);
      const int excl = (int)mbcnt64(c1) + 2 * (int)mbcnt64(c2) + 4 * (int)mbcnt64(c4);
      const int total = __popcll(c1) + 2 * __popcll(c2) + 4 * __popcll(c4);
      const unsigned long long miss = hit_key(__builtin_huge_valf(), -1);
      unsigned long long mine = miss;
      if (n_own > 0) {
        if (!any && h.id >= 0) mine = hit_key(h.t, h.id);
        lf->key[lane] = mine;
        // pair excl + j of this lane, j < n_own, is owned by it.  The lanes
        // with pairs have increasing excl, so no two of them store to one
        // entry in the same store; storing from the last j down, an entry
        // past this lane's count that belongs to a later lane is stored again
        // by that lane (with a smaller j) afterwards, and the entries past the
        // last pair are never read.  The result rests on the order of the
        // stores, which a single-lane view of the code does not see (four
        // stores to distinct bytes), so a wave barrier, which memory
        // operations may not cross, separates them: the compiler can neither
        // reorder nor merge them
#pragma unroll
        for (int j = kLeafMax - 1; j >= 0; --j) {
          lf->owner[excl + j] = (uint8_t)lane;
          __builtin_amdgcn_wave_barrier();
        }
      }
      // pair p of this lane is triangle first + p - excl
      const int tri_base = first - excl;
      const float tlim = tmax;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const unsigned long long act = __ballot(1);
      const int n_act = __popcll(act), rank = (int)mbcnt64(act);
      for (int p0 = 0; p0 < total; p0 += n_act) {
        const int p = p0 + rank;
        if (COUNT && first_active_lane()) cnt.wave_tri_iters++;
        // every active lane takes part in the permutes (a lane outside the
        // exec mask supplies no data, and an owner may have no pair of its own
        // this round), and a lane past the last pair repeats the last one, so
        // the triangle loads are issued before the ray permutes they overlap
        const int pc = min(p, total - 1);
        const int src = (int)lf->owner[pc] << 2;  // owner's permute address
        const int i = __builtin_amdgcn_ds_bpermute(src, tri_base) + pc;
        const float4* tp = reinterpret_cast<const float4*>(tris + i);
        const float4 p0v = tp[0], p1v = tp[1];
        const float2 p2v = *reinterpret_cast<const float2*>(tp + 2);
        const V3 qo = mk(bperm(src, om.x), bperm(src, om.y), bperm(src, om.z));
        const V3 qd = mk(bperm(src, dm.x), bperm(src, dm.y), bperm(src, dm.z));
        const float qt = bperm(src, tlim);
        if (p < total) {
          if (COUNT) cnt.tris++;
          float t;
          const bool hit = hit_tri(qo, qd, mk(p0v.x, p0v.y, p0v.z), mk(p0v.w, p1v.x, p1v.y),
                                   mk(p1v.z, p1v.w, p2v.x), qt, &t);
          atomicMin(&lf->key[src >> 2], hit ? hit_key(t, __float_as_int(p2v.y)) : miss);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (n_own > 0) {
        const unsigned long long best = lf->key[lane];
        if (best != mine) {
          h.t = __uint_as_float((uint32_t)(best >> 32));
          h.id = (int)(uint32_t)best;
          if (any) return true;
        }
      }
    }
    if (node < 0 && sp == 0) {  // instance done: next one, or the query is answered
      inst = next_inst(S, inst + 1);
      if (inst >= S.n_inst) return true;
      to_instance<ROT>(S, inst, o, d, om, dm);
      if (ROT) inv = mk(safe_inv(dm.x), safe_inv(dm.y), safe_inv(dm.z));
      oi = mk(-om.x * inv.x, -om.y * inv.y, -om.z * inv.z);
      stack[0] = S.inst_root[inst];
      sp = 1;
    }
    // suspend once the budget is spent or at most PRDPT_TRACE_QUORUM percent of
    // the lanes that entered are still tracing: the current node goes back on
    // the stack
    if (iters >= budget || __popcll(__ballot(1)) * 100 <= entered * PRDPT_TRACE_QUORUM) {
      if (node >= 0) push_entry(node);
      tr.sp = sp;
      tr.inst = inst;
      return false;
    }
  }
}

__device__ __forceinline__ V3 offset_origin(V3 p, V3 n) {
  const float m = fmaxf(fabsf(p.x), fmaxf(fabsf(p.y), fabsf(p.z)));
  const float eps = 1e-4f * fmaxf(1.0f, m);
  return mk(p.x + n.x * eps, p.y + n.y * eps, p.z + n.z * eps);
}

// orthonormal basis around a unit vector (Duff et al., JCGT 2017)
__device__ __forceinline__ void basis(V3 n, V3* b1, V3* b2) {
  const float sign = copysignf(1.0f, n.z);
  // -1 / (sign + n.z), correctly rounded: for a unit n, |sign + n.z| lies in
  // [1, 2] (or is NaN), recip_nr's domain, and negation is exact
  const float a = -recip_nr(sign + n.z);
  const float b = n.x * n.y * a;
  *b1 = mk(1.0f + sign * n.x * n.x * a, sign * b, -sign * n.x);
  *b2 = mk(b, sign + n.y * n.y * a, -n.y);
}

// eta = ei / et (rounded), passed in: the interface is air against the body,
// so it is either 1/ior or ior, both per-material constants
__device__ __forceinline__ float fresnel_dielectric(float cosi, float ei, float et, float eta) {
  const float sin2t = (eta * eta) * (1.0f - cosi * cosi);
  if (sin2t >= 1.0f) return 1.0f;
  // sin2t is a float below 1, so 1 - sin2t >= 2^-24: sqrt_nr's domain
  const float cost = sqrt_nr(1.0f - sin2t);
  const float rs = (ei * cosi - et * cost) / (ei * cosi + et * cost);
  const float rp = (et * cosi - ei * cost) / (et * cosi + ei * cost);
  return 0.5f * (rs * rs + rp * rp);
}

__device__ __forceinline__ uint4 path_words(uint32_t k0, uint32_t k1, int pix, int smp, int pair,
                                            int tag, int slot, int sub) {
  return philox10(make_uint4((uint32_t)pix, (uint32_t)smp, (uint32_t)pair,
                             ((uint32_t)tag << 24) | ((uint32_t)slot << 8) | (uint32_t)sub),
                  k0, k1);
}

constexpr float kInvPi = 0.318309886183790671538f;

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// Five one-wave work-groups per SIMD (20 per CU): at most 96 VGPRs per lane
// (512 / 5, in granules of 8) and at most six 1280-byte LDS allocation units
// (7680 bytes) per work-group, which the render kernels meet with the
// 13-entry LDS part of the traversal stack and scenes of at most one sphere
// (more spheres lower the resident count, which the launch computes from the
// occupancy calculator and the LDS units).
// The fifth wave hides more of each wave's dependent-instruction latency: four
// waves per SIMD (128 VGPRs, 23 LDS stack entries) took 3 % longer on both
// workloads, although the register allocator now spills a few values outside
// the traversal loops.
#ifndef PRDPT_MIN_WAVES_PER_EU
#define PRDPT_MIN_WAVES_PER_EU 5
#endif

// Load the scene constants and the spheres into LDS and apply perturbation k's
// parameter values (one binding per thread; no two bindings share a field).
__device__ __forceinline__ void load_state(SceneLds& S, float* __restrict__ sph,
                                           int* __restrict__ sph_mat,
                                           const SceneHdr* __restrict__ g,
                                           const float* __restrict__ X, int d) {
  const uint32_t* src = reinterpret_cast<const uint32_t*>(static_cast<const SceneLds*>(g));
  uint32_t* dst = reinterpret_cast<uint32_t*>(&S);
  constexpr int words = sizeof(SceneLds) / 4;
  for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
  const int n_sph = g->n_sph;
  for (int i = threadIdx.x; i < 4 * n_sph; i += blockDim.x) sph[i] = g->sph[i >> 2][i & 3];
  for (int i = threadIdx.x; i < n_sph; i += blockDim.x) sph_mat[i] = g->sph_mat[i];
  __syncthreads();
  for (int j = threadIdx.x; j < d; j += blockDim.x) {
    const int kind = g->bind_kind[j], i = g->bind_index[j], c = g->bind_comp[j];
    const float xj = X[j];
    if (kind == PRDPT_BIND_SPHERE) sph[4 * i + c] = g->sph[i][c] + xj;
    else if (kind == PRDPT_BIND_QUAD) S.quad[i][c] = g->quad[i][c] + xj;
    else if (kind == PRDPT_BIND_MESH) S.inst_xlate[i][c] = g->inst_xlate[i][c] + xj;
    else if (kind == PRDPT_BIND_PLIGHT) S.pl[i][c] = g->pl[i][c] + xj;
    else if (kind == PRDPT_BIND_ALBEDO) S.mat_rgb[i][c] = g->mat_rgb[i][c] + xj;
    else if (kind == PRDPT_BIND_MESH_ROT) S.inst_ang[i][c] = g->inst_ang[i][c] + xj;
  }
  if (g->has_rot) {  // uniform: every thread reads the same header
    __syncthreads();
    if ((int)threadIdx.x < S.n_inst) euler_rotation(S.inst_ang[threadIdx.x], S.inst_rot[threadIdx.x]);
  }
  __syncthreads();
}

// Render one 8x8 pixel tile of perturbation k (S already holds the
// perturbation's scene state in LDS).  Writes *partial_slot = sum over the
// tile's pixels of sum_c (I - R)^2 when it is not null (ref must then be set),
// and the tile's pixels into img (image k) when img != nullptr.
//
// The tile's paths (valid pixels x samples) are jobs that the lanes take in
// order whenever they are free; each lane runs its current path as a state
// machine that traces exactly one ray per loop iteration: the extension ray of
// the current vertex, or one next-event shadow ray.  A lane whose path ends
// takes the next job in the same iteration, so lanes neither wait for the
// longest path of the wave nor for the slowest pixel of the tile, and every
// iteration runs the same traversal code.  A finished path adds its radiance
// to its pixel's sum in LDS (pix); when several lanes finish paths of the same
// pixel in one iteration, the lowest lane adds first (each round, an atomic
// minimum over the lane ids elects one lane per pixel).  The wave's execution
// is a function of its inputs alone, so the order of every pixel's additions,
// and the sum, are reproducible, and nothing per path goes to device memory.
// Per sample the radiance terms are added in the same order as a recursive
// implementation (vertex by vertex; point lights, then area lights).
// LG: the tile size as a compile-time log2 (2 or 3), or 0 to read it from the
// scene (the batched kernel and the counting copy); both decode tiles and
// jobs with the same integer arithmetic, so they render a tile identically.
template <bool COUNT, bool ROT, int LG>
__device__ __forceinline__ void render_tile(const SceneLds& S, const float* __restrict__ sph,
                                            const int* __restrict__ sph_mat,
                                            const Node* __restrict__ nodes,
                                            const Tri* __restrict__ tris,
                                            const int32_t* __restrict__ tri_slot, int k, int tile,
                                            int tag,
                                            uint32_t k0, uint32_t k1, const float* __restrict__ ref,
                                            float* __restrict__ img, float* partial_slot,
                                            unsigned long long* __restrict__ counters,
                                            int* __restrict__ stack, float* __restrict__ wsum,
                                            int crn, volatile int* __restrict__ next_job,
                                            LeafLds* __restrict__ lf, PixLds* __restrict__ pix_sum) {
  // the tile: ts x ts pixels (ts = 8, or 4 for images of few tiles and many
  // samples per pixel), tiles in row-major order
  const int lg = LG ? LG : S.tile_log2, ts = 1 << lg;
  const int tiles_x = (S.W + ts - 1) >> lg;
  const int t = threadIdx.x;
  const int tx0 = (tile % tiles_x) << lg, ty0 = (tile / tiles_x) << lg;
  // lane t sums and writes pixel slot t = (lx, ly) of the tile
  const int lx = t & (ts - 1), ly = t >> lg;
  const int x = tx0 + lx, y = ty0 + ly;
  const bool valid = ly < ts && x < S.W && y < S.H;
  const int pix = y * S.W + x;
  // the tile's valid pixels (tw x th) and its jobs: pixel q, sample c + j / nv
  const int tw = min(ts, S.W - tx0), th = min(ts, S.H - ty0);
  const int nv = tw * th;
  const bool full = nv == ts * ts;  // wave-uniform
  // path streams: the two renders of an antithetic pair share stream k / 2
  // (common random numbers); independent renders (crn = 0) use stream k
  const int pair = crn ? k >> 1 : k;
  const int spp = S.spp;
  const int n_lights = S.n_pl + S.n_area;
  const float inv_w = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(S.inv_w)));
  const float inv_h = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(S.inv_h)));
  const bool pow2_w = inv_w != 0.0f, pow2_h = inv_h != 0.0f;
  int* stk = stack + t;
  int ovf[kStackOverflow];  // stack entries beyond the LDS part (deep descents only)
  Counters cnt{0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};

  // path state
  V3 o = mk(0.0f, 0.0f, 0.0f), dir = o, p = o, n = o;
  float tmax = __builtin_huge_valf();
  bool shadow = false, specular = true;
  float b0 = 1.0f, b1 = 1.0f, b2 = 1.0f, L0 = 0.0f, L1 = 0.0f, L2 = 0.0f;
  float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;  // pending next-event contribution
  int v = 0, mat = 0, light = -1;          // light >= 0: next-event stage of a diffuse vertex
  uint4 w = make_uint4(0u, 0u, 0u, 0u);

  // the path in flight: sample jslot >> 6 of the tile pixel in slot
  // jslot & 63 = x + ts y, whose sum is pix_sum entry jslot & 63; -1 when the
  // lane has none
  int jslot = -1;
  bool tracing = false;   // a query is in flight (possibly suspended)
  bool answered = false;  // the last query's result (tr.h) is still to be used
  Trav tr;
  // image pixel index and sample of the path in flight
  auto path_pix = [&]() { return (ty0 + ((jslot & 63) >> lg)) * S.W + tx0 + (jslot & (ts - 1)); };
  auto path_smp = [&]() { return jslot >> 6; };
  const int n_jobs = nv * spp;
  uint32_t* const claim = reinterpret_cast<uint32_t*>(lf->owner);
  pix_sum->rgb[0][t] = 0.0f;
  pix_sum->rgb[1][t] = 0.0f;
  pix_sum->rgb[2][t] = 0.0f;
  if (t == 0) *next_job = 0;
  __syncthreads();
  while (true) {
    if (!tracing) {
      if (answered) {
        answered = false;
        const Hit h = tr.h;
        bool end_path = false;
        if (shadow) {
          if (h.id < 0) {
            L0 = L0 + c0;
            L1 = L1 + c1;
            L2 = L2 + c2;
          }
          ++light;
        } else if (h.id < 0) {
          L0 = L0 + b0 * S.env[0];
          L1 = L1 + b1 * S.env[1];
          L2 = L2 + b2 * S.env[2];
          end_path = true;
        } else {
          p = at(o, dir, h.t);
          V3 ng;
          if (h.id < S.n_sph) {
            mat = sph_mat[h.id];
            ng = unit(sub(p, ld3(sph + 4 * h.id)));
          } else if (h.id < S.tri_id_base) {
            const int qi = h.id - S.n_sph;
            mat = S.quad_mat[qi];
            ng = ld3(S.quad_nu[qi]);
          } else {
            const float4* tp =
                reinterpret_cast<const float4*>(tris + tri_slot[h.id - S.tri_id_base]);
            const float4 p0 = tp[0], p1 = tp[1], p2 = tp[2];
            mat = __float_as_int(p2.z);
            ng = cross(mk(p0.w, p1.x, p1.y), mk(p1.z, p1.w, p2.x));  // the mesh's frame
            // into the world by the instance's rotation; without rotations it
            // is the zero-angle matrix, still applied: its zero entries decide
            // the sign of a zero normal component, and that sign picks the
            // tangent frame of the bounce
            if (ROT) {
              const float* R = S.inst_rot[__float_as_int(p2.w)];
              ng = mk(R[0] * ng.x + R[1] * ng.y + R[2] * ng.z, R[3] * ng.x + R[4] * ng.y + R[5] * ng.z,
                      R[6] * ng.x + R[7] * ng.y + R[8] * ng.z);
            } else {
              ng = mk(ng.x + 0.0f * ng.y + 0.0f * ng.z, 0.0f * ng.x + ng.y + 0.0f * ng.z,
                      0.0f * ng.x + 0.0f * ng.y + ng.z);
            }
            ng = unit(ng);
          }
          const int mt = S.mat_type[mat];
          if (mt == PRDPT_MAT_EMISSIVE) {
            if (specular && dot(dir, ng) < 0.0f) {
              L0 = L0 + b0 * S.mat_rgb[mat][0];
              L1 = L1 + b1 * S.mat_rgb[mat][1];
              L2 = L2 + b2 * S.mat_rgb[mat][2];
            }
            end_path = true;
          } else {
            w = path_words(k0, k1, path_pix(), path_smp(), pair, tag, v + 1, 0);
            if (mt == PRDPT_MAT_DIFFUSE) {
              n = dot(ng, dir) > 0.0f ? neg(ng) : ng;
              light = 0;
            } else if (v == S.B) {  // dielectric sphere, bounce budget spent
              end_path = true;
            } else {
              const float ior = S.mat_ior[mat];
              V3 nn = ng;
              float cosi = -dot(dir, nn);
              float ei = 1.0f, et = ior;
              float eta = S.mat_rgb[mat][0];  // 1 / ior: entering the body
              if (cosi < 0.0f) {
                nn = neg(nn);
                cosi = -cosi;
                ei = ior;
                et = 1.0f;
                eta = ior;  // ior / 1: leaving it
              }
              const float F = fresnel_dielectric(cosi, ei, et, eta);
              V3 nd, side;
              if (unit_open(w.z) < F) {
                const float dn = dot(dir, nn);
                nd = mk(dir.x - nn.x * (2.0f * dn), dir.y - nn.y * (2.0f * dn), dir.z - nn.z * (2.0f * dn));
                side = nn;
              } else {
                const float sin2t = (eta * eta) * (1.0f - cosi * cosi);
                // refraction only when F < 1, i.e. sin2t < 1: 1 - sin2t >= 2^-24
                const float cost = sqrt_nr(1.0f - sin2t);
                const float kk = eta * cosi - cost;
                nd = mk(dir.x * eta + nn.x * kk, dir.y * eta + nn.y * kk, dir.z * eta + nn.z * kk);
                side = neg(nn);
              }
              o = offset_origin(p, side);
              dir = unit(nd);
              tmax = __builtin_huge_valf();
              specular = true;
              ++v;
            }
          }
        }
        if (!end_path && light >= 0) {
          // next-event estimation at a diffuse vertex: set up the next light whose
          // sample faces both surfaces, else continue the path
          shadow = false;
          const float f0 = S.mat_rgb[mat][0] * kInvPi, f1 = S.mat_rgb[mat][1] * kInvPi,
                      f2 = S.mat_rgb[mat][2] * kInvPi;
          for (; light < n_lights; ++light) {
            if (light < S.n_pl) {
              const float* lp = S.pl[light];
              const V3 toL = sub(ld3(lp), p);
              const float dist2 = dot(toL, toL);
              const float dist = sqrt_cr(dist2);
              const V3 wi = scale(toL, recip_nr(dist));  // dist: a root, as in unit()
              const float cx = dot(n, wi);
              if (!(cx > 0.0f)) continue;
              c0 = b0 * f0 * ((lp[3] * cx) / dist2);
              c1 = b1 * f1 * ((lp[4] * cx) / dist2);
              c2 = b2 * f2 * ((lp[5] * cx) / dist2);
              o = offset_origin(p, n);
              dir = wi;
              tmax = dist * 0.9999f;
              shadow = true;
              break;
            }
            const int ai = light - S.n_pl;
            const int qi = S.area_quad[ai];
            float ua, ub;
            if (ai == 0) {
              ua = unit_open(w.x);
              ub = unit_open(w.y);
            } else {
              const uint4 w2 = path_words(k0, k1, path_pix(), path_smp(), pair, tag, v + 1, ai);
              ua = unit_open(w2.x);
              ub = unit_open(w2.y);
            }
            const float* qd = S.quad[qi];
            const V3 qo = ld3(qd), e1 = ld3(qd + 3), e2 = ld3(qd + 6);
            const V3 yl = mk(qo.x + e1.x * ua + e2.x * ub, qo.y + e1.y * ua + e2.y * ub,
                             qo.z + e1.z * ua + e2.z * ub);
            const V3 nlu = ld3(S.quad_nu[qi]);
            const float area = S.quad_nu[qi][3];
            const V3 toL = sub(yl, p);
            const float dist2 = dot(toL, toL);
            const float dist = sqrt_cr(dist2);
            const V3 wi = scale(toL, recip_nr(dist));  // dist: a root, as in unit()
            const float cx = dot(n, wi);
            const float cl = -dot(nlu, wi);
            if (!(cx > 0.0f && cl > 0.0f)) continue;
            const float G = ((cx * cl) * area) / dist2;
            const int qm = S.quad_mat[qi];
            c0 = b0 * f0 * S.mat_rgb[qm][0] * G;
            c1 = b1 * f1 * S.mat_rgb[qm][1] * G;
            c2 = b2 * f2 * S.mat_rgb[qm][2] * G;
            o = offset_origin(p, n);
            dir = wi;
            tmax = dist * 0.9999f;
            shadow = true;
            break;
          }
          if (!shadow) {  // all lights done: cosine-weighted bounce
            light = -1;
            if (v == S.B) {
              end_path = true;
            } else {
              const float u1 = unit_open(w.z), u2 = unit_open(w.w);
              // u1 and 1 - u1 lie in [2^-24, 1]: sqrt_nr's domain
              const float r = sqrt_nr(u1);
              float sn, cs;
              sincos_turn(u2, &sn, &cs);
              const float lx2 = r * cs, ly2 = r * sn, lz2 = sqrt_nr(1.0f - u1);
              V3 e1, e2;
              basis(n, &e1, &e2);
              dir = unit(mk(e1.x * lx2 + e2.x * ly2 + n.x * lz2, e1.y * lx2 + e2.y * ly2 + n.y * lz2,
                            e1.z * lx2 + e2.z * ly2 + n.z * lz2));
              o = offset_origin(p, n);
              tmax = __builtin_huge_valf();
              b0 = b0 * S.mat_rgb[mat][0];
              b1 = b1 * S.mat_rgb[mat][1];
              b2 = b2 * S.mat_rgb[mat][2];
              specular = false;
              ++v;
            }
          }
        }
        // finished paths add their radiance to their pixels' sums; lanes with
        // the same pixel take turns, lowest lane first
        const int q = jslot & (kBlock - 1);
        bool deposit = end_path;
        while (__ballot(deposit) != 0ull) {
          if (deposit) claim[q] = 0xffffffffu;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          if (deposit) atomicMin(&claim[q], (uint32_t)t);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          if (deposit && claim[q] == (uint32_t)t) {
            pix_sum->rgb[0][q] = pix_sum->rgb[0][q] + L0;
            pix_sum->rgb[1][q] = pix_sum->rgb[1][q] + L1;
            pix_sum->rgb[2][q] = pix_sum->rgb[2][q] + L2;
            deposit = false;
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (end_path) jslot = -1;
      }
      if (jslot < 0) {  // the lanes without a path take the tile's next jobs in order
        const unsigned long long m = __ballot(1);
        const int rank = (int)__builtin_amdgcn_mbcnt_hi(
            (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        // one read of the wave's job counter, broadcast, then the update: the
        // update depends on the value read, so no lane can see it early,
        // however the compiler lays out the branch
        const int base = __builtin_amdgcn_readfirstlane(*next_job);
        const int j = base + rank;
        __builtin_amdgcn_wave_barrier();
        if (rank == 0) *next_job = base + __popcll(m);
        if (j >= n_jobs) break;  // this lane is done with the tile
        const int q = full ? (j & (nv - 1)) : j % nv;
        const int sj = full ? (j >> (2 * lg)) : j / nv;
        const int qx = tw == ts ? (q & (ts - 1)) : q % tw;
        const int qy = tw == ts ? (q >> lg) : q / tw;
        jslot = sj * kBlock + qx + (qy << lg);
        // camera ray of the path
        if (COUNT) cnt.paths++;
        float jxo = 0.5f, jyo = 0.5f;
        if (!S.pixel_center) {
          const uint4 wj = path_words(k0, k1, path_pix(), path_smp(), pair, tag, 0, 0);
          jxo = unit_open(wj.x);
          jyo = unit_open(wj.y);
        }
        const float px = (float)(tx0 + qx) + jxo, py = (float)(ty0 + qy) + jyo;
        // dividing by a power of two is exact, and so is multiplying by its
        // inverse (a wave-uniform choice)
        const float sx = 2.0f * (pow2_w ? px * inv_w : px / (float)S.W) - 1.0f;
        const float sy = 1.0f - 2.0f * (pow2_h ? py * inv_h : py / (float)S.H);
        o = ld3(S.eye);
        dir = unit(mk(S.fwd[0] + S.right[0] * sx + S.up[0] * sy,
                      S.fwd[1] + S.right[1] * sx + S.up[1] * sy,
                      S.fwd[2] + S.right[2] * sx + S.up[2] * sy));
        tmax = __builtin_huge_valf();
        shadow = false;
        specular = true;
        b0 = b1 = b2 = 1.0f;
        L0 = L1 = L2 = 0.0f;
        v = 0;
        light = -1;
      }
      tracing = !begin_trace<COUNT>(S, sph, o, dir, tmax, shadow, tr, stk, cnt);
      if (!tracing) {
        answered = true;
        continue;
      }
    }
    if (COUNT) {
      const int active = __popcll(__ballot(1));
      if (first_active_lane()) {
        cnt.wave_outer_iters++;
        cnt.idle_lane_iters += 64 - active;
      }
    }
    tracing = !continue_trace<COUNT, ROT>(S, nodes, tris, o, dir, tmax, shadow, tr, stk, kBlock,
                                          ovf, lf, PRDPT_TRACE_BUDGET, cnt);
    answered = !tracing;
  }
  // every path of the tile is done: lane t reads pixel t's sum
  __syncthreads();
  float e = 0.0f;
  if (valid) {
    const float inv_spp = 1.0f / (float)spp;
    const float I0 = pix_sum->rgb[0][t] * inv_spp, I1 = pix_sum->rgb[1][t] * inv_spp,
                I2 = pix_sum->rgb[2][t] * inv_spp;
    const size_t npix = (size_t)S.W * S.H;
    if (img) {
      float* op = img + ((size_t)k * npix + pix) * 3;
      op[0] = I0;
      op[1] = I1;
      op[2] = I2;
    }
    if (ref) {
      const float* r = ref + (size_t)pix * 3;
      const float d0 = I0 - r[0], d1 = I1 - r[1], d2 = I2 - r[2];
      e = d0 * d0 + d1 * d1 + d2 * d2;
    }
  }
  if (COUNT) {
    atomicAdd(&counters[0], (unsigned long long)cnt.nodes);
    atomicAdd(&counters[1], (unsigned long long)cnt.tris);
    atomicAdd(&counters[2], (unsigned long long)cnt.rays);
    atomicAdd(&counters[3], (unsigned long long)cnt.paths);
    atomicAdd(&counters[4], (unsigned long long)cnt.wave_node_iters);
    atomicAdd(&counters[5], (unsigned long long)cnt.wave_tri_iters);
    atomicAdd(&counters[6], (unsigned long long)cnt.wave_outer_iters);
    atomicAdd(&counters[7], (unsigned long long)cnt.idle_lane_iters);
    atomicAdd(&counters[8], (unsigned long long)cnt.overflow_pushes);
    atomicMax(&counters[9], (unsigned long long)cnt.deepest);
  }
  if (partial_slot) {
    // fixed-order butterfly within the wave, then the waves in order
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
    if ((t & 63) == 0) wsum[t >> 6] = e;
    __syncthreads();
    if (t == 0) {
      float sum = wsum[0];
      for (int wv = 1; wv < kBlock / 64; ++wv) sum = sum + wsum[wv];
      *partial_slot = sum;
    }
  }
}


// Single-request launch, persistent: a grid of at most the resident work-group
// count whose work-groups take (perturbation k, tile) items in order from the
// counter *work (zeroed by reset_work_kernel before the launch) until all
// n_tiles * nk items are done.  Dynamic assignment keeps every CU busy when
// tiles differ widely in cost, where a one-work-group-per-tile grid leaves
// CUs idle waiting on the hardware dispatcher.  Within each perturbation the
// tiles are taken in the order order[] (null: index order), and each tile's
// render time is stored in cost[tile] (when not null), so that sorting the
// tiles by cost for the next launch puts the cheapest tiles last and shortens
// the tail where few work-groups are still busy.  Outputs do not depend on
// the order.
template <bool COUNT, bool ROT, int LG>
__global__ __launch_bounds__(kBlock, PRDPT_MIN_WAVES_PER_EU) void render_loss_kernel(
    DevScene scene, const float* __restrict__ X, int d, int tag, uint32_t k0, uint32_t k1,
    const float* __restrict__ ref, float* __restrict__ img, float* __restrict__ partial,
    unsigned long long* __restrict__ counters, int n_tiles, int n_items, int* __restrict__ work,
    const int* __restrict__ order, float* __restrict__ cost, int crn) {
  __shared__ SceneLds S;
  __shared__ int stack[kStackEntries * kBlock];
  __shared__ float wsum[kBlock / 64];
  __shared__ int s_item;
  __shared__ int s_job;
  __shared__ LeafLds s_leaf;
  __shared__ PixLds s_pix;
  extern __shared__ float sph[];  // sphere_lds_bytes(n_sph) at launch
  int* sph_mat = reinterpret_cast<int*>(sph + 4 * scene.hdr->n_sph);
  int cur = -1;
  while (true) {
    if (threadIdx.x == 0) s_item = atomicAdd(work, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= n_items) break;
    const int k = it / n_tiles, j = it - k * n_tiles;
    int tile = order ? order[j] : j;
    if ((unsigned)tile >= (unsigned)n_tiles) tile = j;  // a permutation by construction
    if (k != cur) {  // the scene state of perturbation k (after the previous tile's last use)
      load_state(S, sph, sph_mat, scene.hdr, X + (size_t)k * d, d);
      cur = k;
    }
    unsigned long long t0 = 0;
    if (cost && threadIdx.x == 0) t0 = wall_clock64();
    render_tile<COUNT, ROT, LG>(S, sph, sph_mat, scene.nodes, scene.tris, scene.tri_slot, k, tile,
                       tag, k0, k1, ref, img,
                       partial ? partial + (size_t)k * n_tiles + tile : nullptr, counters, stack,
                       wsum, crn, &s_job, &s_leaf, &s_pix);
    if (cost && threadIdx.x == 0) cost[tile] = (float)(wall_clock64() - t0);
    __syncthreads();
  }
}

__global__ void reset_work_kernel(int* __restrict__ work) {
  if (threadIdx.x == 0) work[0] = 0;
}

// order[0..n) = tile indices by descending cost (bitonic sort of at most
// kOrderMax keys in LDS by one work-group; ties in an arbitrary fixed order)
constexpr int kOrderMax = 4096;
__global__ __launch_bounds__(1024) void tile_order_kernel(const float* __restrict__ cost,
                                                          int* __restrict__ order, int n) {
  __shared__ float key[kOrderMax];
  __shared__ int val[kOrderMax];
  int m = 1;
  while (m < n) m <<= 1;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    key[i] = i < n ? cost[i] : -1.0f;  // costs are >= 0: padding sorts last
    val[i] = i;
  }
  __syncthreads();
  for (int size = 2; size <= m; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const int jx = i ^ stride;
        if (jx > i) {
          const bool down = (i & size) == 0;  // blocks alternate; the last merge is descending
          const float ki = key[i], kj = key[jx];
          if (down ? (ki < kj) : (ki > kj)) {
            key[i] = kj;
            key[jx] = ki;
            const int t = val[i];
            val[i] = val[jx];
            val[jx] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) order[i] = val[i];
}

// Perturbation draw for pair p (Sec. 3.2): Philox TAU stream words in order,
// tau_p, binary64 pair weights c_p, and the parameter rows theta +- tau_p
// (Xm null: draw p of independent perturbations, row theta + tau_p only).
// Rows are written with stride `ld` (>= d).
__device__ void draw_pair(int est, int d, int p, uint32_t k0, uint32_t k1,
                          const float* __restrict__ sigma, const float* __restrict__ theta,
                          double cd, double sqrt2pi, int ld, float* __restrict__ tau,
                          double* __restrict__ c, float* __restrict__ Xp, float* __restrict__ Xm,
                          int strata) {
  uint32_t blk = 0;
  int used = 4;
  uint4 w = make_uint4(0, 0, 0, 0);
  auto word = [&]() -> uint32_t {
    if (used == 4) {
      w = philox10(make_uint4((uint32_t)p, blk, 0u, (uint32_t)kTagTau << 24), k0, k1);
      ++blk;
      used = 0;
    }
    const uint32_t r = used == 0 ? w.x : used == 1 ? w.y : used == 2 ? w.z : w.w;
    ++used;
    return r;
  };
  // the draw's next uniform; with strata > 0 the first one is moved into
  // stratum p of strata, (p + u) / strata, kept below 1
  bool to_stratify = strata > 0;
  auto uniform = [&]() -> float {
    float u = unit_open(word());
    if (to_stratify) {
      u = fminf(((float)p + u) / (float)strata, 0x1.fffffep-1f);
      to_stratify = false;
    }
    return u;
  };
  auto gauss2 = [&](float* z0, float* z1) {
    const float u1 = uniform();
    const float u2 = uniform();
    const float rad = sqrtf(-2.0f * log_ieee(u1));
    float sn, cs;
    sincos_turn(u2, &sn, &cs);
    *z0 = rad * cs;
    *z1 = rad * sn;
  };
  // without antithetic partners each draw carries the single-sample score
  // weight, twice the pair weight (exact in binary64).  The row tau holds the
  // normal or radius draws until their final values replace them.
  const double wscale = (est & PRDPT_EST_INDEPENDENT) ? 2.0 : 1.0;
  est &= ~(PRDPT_EST_INDEPENDENT | PRDPT_EST_STRATIFIED);
  if (est == PRDPT_EST_GAUSS) {
    for (int j = 0; j < d; j += 2) {
      float z0, z1;
      gauss2(&z0, &z1);
      tau[j] = z0;
      if (j + 1 < d) tau[j + 1] = z1;
    }
    for (int j = 0; j < d; ++j) {
      const float v = tau[j];
      tau[j] = sigma[j] * v;
      c[j] = wscale * ((double)v / (2.0 * (double)sigma[j]));
    }
  } else if (est == PRDPT_EST_IS) {
    const int m = (d + 1) / 2;
    float acc = 0.0f;
    for (int i = 0; i < m; ++i) acc = acc + log_ieee(uniform());
    float rho2 = -2.0f * acc;
    if ((d + 1) & 1) {
      float z0, z1;
      gauss2(&z0, &z1);
      rho2 = rho2 + z0 * z0;
    }
    for (int j = 0; j < d; j += 2) {
      float z0, z1;
      gauss2(&z0, &z1);
      tau[j] = z0;
      if (j + 1 < d) tau[j + 1] = z1;
    }
    float n2 = 0.0f;
    for (int j = 0; j < d; ++j) n2 = n2 + tau[j] * tau[j];
    const float nrm = sqrtf(n2);
    const float rho = sqrtf(rho2);
    for (int j = 0; j < d; ++j) {
      const float uj = tau[j] / nrm;
      tau[j] = sigma[j] * (rho * uj);
      c[j] = wscale * (cd * (double)uj / (2.0 * (double)sigma[j]));
    }
  } else {
    for (int j = 0; j < d; ++j) tau[j] = sqrtf(-2.0f * log_ieee(uniform()));
    uint32_t bits = 0;
    for (int j = 0; j < d; ++j) {  // one sign word per 32 axes, after the radii
      if ((j & 31) == 0) bits = word();
      const float sg = ((bits >> (j & 31)) & 1u) ? -1.0f : 1.0f;
      tau[j] = sigma[j] * (sg * tau[j]);
      c[j] = wscale * ((double)sg / ((double)sigma[j] * sqrt2pi));
    }
  }
  for (int j = 0; j < d; ++j) {
    Xp[j] = theta[j] + tau[j];
    if (Xm) Xm[j] = theta[j] - tau[j];
  }
  (void)ld;
}

// Per-image loss: (sum of the image's tile partials) / (3 H W) in binary64, one
// wave per image, lane i summing tiles i, i+64, ..., then a fixed butterfly.
__device__ __forceinline__ double row_loss(const float* __restrict__ part, int n_tiles,
                                           double inv_den) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int i = lane; i < n_tiles; i += 64) s += (double)part[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s * inv_den;
}

// g_j = scale (1/P) sum_p c_pj (L_2p - L_2p+1) and Q = mean L, binary64, pair
// order (Eq. 10 with antithetic pairs); c rows have stride ld.  Thread t takes
// the components t, t + blockDim.x, ...
__device__ __forceinline__ void combine_one(int P, int d, int ld, const double* __restrict__ c,
                                            const double* __restrict__ L, double sc,
                                            double* __restrict__ grad, double* __restrict__ loss) {
  for (int j = threadIdx.x; j < d; j += blockDim.x) {
    double acc = 0.0;
    for (int p = 0; p < P; ++p) acc += c[(size_t)p * ld + j] * (L[2 * p] - L[2 * p + 1]);
    grad[j] = sc * (acc / (double)P);
  }
  if (threadIdx.x == 0 && loss) {
    double s = 0.0;
    for (int k = 0; k < 2 * P; ++k) s += L[k];
    *loss = s / (double)(2 * P);
  }
}

// Independent perturbations: g_j = scale (1/N) sum_i c_ij L_i, Q = mean L.
__device__ __forceinline__ void combine_independent(int N, int d, const double* __restrict__ c,
                                                    const double* __restrict__ L, double sc,
                                                    double* __restrict__ grad,
                                                    double* __restrict__ loss) {
  for (int j = threadIdx.x; j < d; j += blockDim.x) {
    double acc = 0.0;
    for (int i = 0; i < N; ++i) acc += c[(size_t)i * d + j] * L[i];
    grad[j] = sc * (acc / (double)N);
  }
  if (threadIdx.x == 0 && loss) {
    double s = 0.0;
    for (int i = 0; i < N; ++i) s += L[i];
    *loss = s / (double)N;
  }
}

// One thread per antithetic pair: tau_p, weights c_p and the two parameter rows
// (or, with PRDPT_EST_INDEPENDENT, one thread per independent draw, whose first
// uniforms are stratified over the P draws with PRDPT_EST_STRATIFIED).
__global__ void tau_kernel(int est, int d, int P, uint32_t k0, uint32_t k1,
                           const float* __restrict__ sigma, const float* __restrict__ theta,
                           double cd, double sqrt2pi, float* __restrict__ tau,
                           double* __restrict__ c, float* __restrict__ X) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  if (est & PRDPT_EST_INDEPENDENT)  // P independent draws, one parameter row each
    draw_pair(est, d, p, k0, k1, sigma, theta, cd, sqrt2pi, d, tau + (size_t)p * d,
              c + (size_t)p * d, X + (size_t)p * d, nullptr,
              (est & PRDPT_EST_STRATIFIED) ? P : 0);
  else
    draw_pair(est, d, p, k0, k1, sigma, theta, cd, sqrt2pi, d, tau + (size_t)p * d,
              c + (size_t)p * d, X + (size_t)(2 * p) * d, X + (size_t)(2 * p + 1) * d, 0);
}

__global__ void loss_kernel(const float* __restrict__ partial, int n_tiles, int N, double inv_den,
                            double* __restrict__ losses) {
  const int k = blockIdx.x;
  const double L = row_loss(partial + (size_t)k * n_tiles, n_tiles, inv_den);
  if (threadIdx.x == 0) losses[k] = L;
}

__global__ void combine_kernel(int rows, int d, int independent, const double* __restrict__ c,
                               const double* __restrict__ L, const double* __restrict__ scale,
                               double* __restrict__ grad, double* __restrict__ loss) {
  if (independent)
    combine_independent(rows, d, c, L, scale ? *scale : 1.0, grad, loss);
  else
    combine_one(rows, d, d, c, L, scale ? *scale : 1.0, grad, loss);
}

// ---------------------------------------------------------------------------
// batched form: many requests (different scenes, sizes, N, d) in one pass.
// Every per-request result is computed by the same device functions in the same
// order as the single-request kernels, so it is bit-identical to running the
// request alone.
// ---------------------------------------------------------------------------
// index of the last request whose field (int at byte offset `off`) is <= key
__device__ __forceinline__ int find_request(const BatchReq* __restrict__ reqs, int n, int key,
                                            size_t off) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int v = *reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(reqs + mid) + off);
    if (v <= key) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void batch_reset_kernel(BatchMeta* meta) {
  if (threadIdx.x == 0 && blockIdx.x == 0) meta->counter = 0;
}

__global__ void batch_tau_kernel(const BatchReq* __restrict__ reqs, const BatchMeta* __restrict__ meta,
                                 float* __restrict__ tau, double* __restrict__ c,
                                 float* __restrict__ X) {
  const int total = meta->total_pairs, n = meta->n_req;
  constexpr int ld = PRDPT_BATCH_MAX_PARAMS;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < total; g += gridDim.x * blockDim.x) {
    const int r = find_request(reqs, n, g, offsetof(BatchReq, pair_base));
    const BatchReq& q = reqs[r];
    const int p = g - q.pair_base;
    draw_pair(q.est, q.d, p, q.k0, q.k1, q.sigma, q.theta, q.cd, q.sqrt2pi, ld,
              tau + (size_t)g * ld, c + (size_t)g * ld, X + (size_t)(q.row_base + 2 * p) * ld,
              X + (size_t)(q.row_base + 2 * p + 1) * ld, 0);
  }
}

// Persistent render: work-groups take (request, perturbation, run of tiles)
// items from one counter until the batch is exhausted; each tile writes its own
// partial slot, so the order in which items are taken does not matter.
template <bool ROT>
__global__ __launch_bounds__(kBlock, PRDPT_MIN_WAVES_PER_EU) void batch_render_kernel(
    const BatchReq* __restrict__ reqs, BatchMeta* __restrict__ meta, const float* __restrict__ X,
    float* __restrict__ partial) {
  __shared__ SceneLds S;
  __shared__ int stack[kStackEntries * kBlock];
  __shared__ float wsum[kBlock / 64];
  __shared__ int s_item;
  __shared__ int s_job;
  __shared__ LeafLds s_leaf;
  __shared__ PixLds s_pix;
  extern __shared__ float sph[];  // sphere_lds_bytes(largest n_sph of the batch) at launch
  const int total = meta->total_items, n = meta->n_req, tpi = meta->tiles_per_item;
  while (true) {
    if (threadIdx.x == 0) s_item = atomicAdd(&meta->counter, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= total) break;
    const int r = find_request(reqs, n, it, offsetof(BatchReq, item_base));
    const BatchReq& q = reqs[r];
    const int local = it - q.item_base;
    const int k = local / q.items_per_row;
    const int first = (local % q.items_per_row) * tpi;
    const int last = min(first + tpi, q.n_tiles);
    int* sph_mat = reinterpret_cast<int*>(sph + 4 * q.scene.hdr->n_sph);
    load_state(S, sph, sph_mat, q.scene.hdr, X + (size_t)(q.row_base + k) * PRDPT_BATCH_MAX_PARAMS,
               q.d);
    for (int tile = first; tile < last; ++tile) {
      render_tile<false, ROT, 0>(S, sph, sph_mat, q.scene.nodes, q.scene.tris, q.scene.tri_slot, k,
                         tile, kTagPath, q.k0, q.k1, q.ref,
                         nullptr, partial + (size_t)q.partial_base + (size_t)k * q.n_tiles + tile,
                         nullptr, stack, wsum, 1, &s_job, &s_leaf, &s_pix);
      __syncthreads();
    }
  }
}

__global__ void batch_loss_kernel(const BatchReq* __restrict__ reqs,
                                  const BatchMeta* __restrict__ meta,
                                  const float* __restrict__ partial, double* __restrict__ losses) {
  const int total = meta->total_rows, n = meta->n_req;
  for (int g = blockIdx.x; g < total; g += gridDim.x) {
    const int r = find_request(reqs, n, g, offsetof(BatchReq, row_base));
    const BatchReq& q = reqs[r];
    const int k = g - q.row_base;
    const double L = row_loss(partial + (size_t)q.partial_base + (size_t)k * q.n_tiles, q.n_tiles,
                              q.inv_den);
    if (threadIdx.x == 0) losses[g] = L;
  }
}

__global__ void batch_combine_kernel(const BatchReq* __restrict__ reqs,
                                     const BatchMeta* __restrict__ meta,
                                     const double* __restrict__ c, const double* __restrict__ losses,
                                     double* __restrict__ grads, double* __restrict__ loss) {
  for (int r = blockIdx.x; r < meta->n_req; r += gridDim.x) {
    const BatchReq& q = reqs[r];
    combine_one(q.N / 2, q.d, PRDPT_BATCH_MAX_PARAMS,
                c + (size_t)q.pair_base * PRDPT_BATCH_MAX_PARAMS, losses + q.row_base, 1.0,
                grads + (size_t)r * PRDPT_BATCH_MAX_PARAMS, loss + r);
  }
}

// Plain streaming copy (16-byte loads and stores, grid-stride): the reference
// for achievable HBM bandwidth and for scaling the memory counters.
// Every binary32 x in [base, base + n) (as bit patterns): each fast
// correctly rounded operation of exact_math.h against the compiler's correctly
// rounded one, on the inputs of its stated domain; a NaN equals any NaN.
// bad[0..2]: recip_nr, sqrt_nr, sqrt_cr mismatches.
__device__ __forceinline__ bool same_value(float a, float b) {
  return (a != a && b != b) || __float_as_uint(a) == __float_as_uint(b);
}
__global__ __launch_bounds__(256) void math_selftest_kernel(uint32_t base, uint32_t n,
                                                            unsigned long long* __restrict__ bad) {
  uint32_t c0 = 0, c1 = 0, c2 = 0;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float x = __uint_as_float(base + i);
    const float ax = fabsf(x);
    const float q = 1.0f / x, r = sqrtf(x);
    const bool rdom = ax <= 0x1p126f ? (ax >= 0x1p-126f || ax == 0.0f) : !(ax < __builtin_huge_valf());
    c0 += rdom && !same_value(recip_nr(x), q);
    const bool sdom = !(ax > 0.0f && ax < 0x1p-104f);
    c1 += sdom && !same_value(sqrt_nr(x), r);
    c2 += !same_value(sqrt_cr(x), r);
    if (i > 0xffffffffu - stride) break;  // the next index would wrap
  }
  if (c0) atomicAdd(&bad[0], (unsigned long long)c0);
  if (c1) atomicAdd(&bad[1], (unsigned long long)c1);
  if (c2) atomicAdd(&bad[2], (unsigned long long)c2);
}

__global__ __launch_bounds__(256) void copy_kernel(const float4* __restrict__ src,
                                                   float4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Eq. 9: the kernel-smoothed gradient of a differentiable renderer, for
// scenes of one diffuse sphere (its centre bound) over one diffuse ground quad
// under one point light, direct light only.  The pixel derivative is the
// interior term (the sphere's shading moves with its centre) plus samples on
// the two moving edges, the silhouette and the shadow boundary, each the image
// of a circle of tangent points; every term is weighted here by the pixel's
// (I - R) and summed, giving the loss gradient of one render.
// ---------------------------------------------------------------------------
constexpr int kTagDiff = 6, kTagEdge = 7;

// one render's sphere (centre, radius), its parameter rows applied
struct DpState {
  V3 c;
  float rho;
  const SceneHdr* g;
};

__device__ __forceinline__ DpState dp_state(const SceneHdr* __restrict__ g, const float* __restrict__ X,
                                            int d) {
  float c3[3] = {g->sph[0][0], g->sph[0][1], g->sph[0][2]};
  for (int j = 0; j < d; ++j) {
    const int ax = g->bind_comp[j];
    c3[ax] = g->sph[0][ax] + X[j];
  }
  return DpState{mk(c3[0], c3[1], c3[2]), g->sph[0][3], g};
}

// pixel position of world point P and the rows of d(px, py)/dP
__device__ __forceinline__ void dp_project(const SceneHdr* __restrict__ g, V3 P, float* px, float* py,
                                           V3* jx, V3* jy) {
  const V3 e = ld3(g->eye), f = ld3(g->fwd), r = ld3(g->right), u = ld3(g->up);
  const V3 D = sub(P, e);
  const float lam = dot(D, f), a = dot(D, r), b = dot(D, u);
  const float rr = dot(r, r), uu = dot(u, u);
  const float sx = a / (lam * rr), sy = b / (lam * uu);
  const float hw = 0.5f * (float)g->W, hh = 0.5f * (float)g->H;
  *px = (sx + 1.0f) * hw;
  *py = (1.0f - sy) * hh;
  const float l2r = (lam * lam) * rr, l2u = (lam * lam) * uu;
  const V3 gx = mk((r.x * lam - f.x * a) / l2r, (r.y * lam - f.y * a) / l2r, (r.z * lam - f.z * a) / l2r);
  const V3 gy = mk((u.x * lam - f.x * b) / l2u, (u.y * lam - f.y * b) / l2u, (u.z * lam - f.z * b) / l2u);
  *jx = scale(gx, hw);
  *jy = scale(gy, -hh);
}

// direct radiance of a diffuse point under the point light, no shadow test
__device__ __forceinline__ void dp_shade(const SceneHdr* __restrict__ g, int mat, V3 p, V3 n, float out[3]) {
  const float* lp = g->pl[0];
  const V3 toL = sub(ld3(lp), p);
  const float dist2 = dot(toL, toL);
  const float dist = sqrtf(dist2);
  const V3 wi = scale(toL, 1.0f / dist);
  const float cx = dot(n, wi);
  for (int c = 0; c < 3; ++c)
    out[c] = cx > 0.0f ? (g->mat_rgb[mat][c] * kInvPi) * ((lp[3 + c] * cx) / dist2) : 0.0f;
}

__device__ __forceinline__ V3 dp_ground_normal(const SceneHdr* __restrict__ g) {
  V3 n = unit(cross(ld3(g->quad[0] + 3), ld3(g->quad[0] + 6)));
  if (dot(n, sub(ld3(g->pl[0]), ld3(g->quad[0]))) < 0.0f) n = neg(n);
  return n;
}

__device__ __forceinline__ float dp_sphere4(const DpState& st, float* sp) {
  sp[0] = st.c.x;
  sp[1] = st.c.y;
  sp[2] = st.c.z;
  sp[3] = st.rho;
  return st.rho;
}

// radiance behind the silhouette: the ground (shadowed or not) or the environment
__device__ __forceinline__ void dp_behind(const DpState& st, V3 o, V3 d, float out[3]) {
  const SceneHdr* g = st.g;
  float t;
  if (!hit_quad(o, d, g->quad[0], g->quad_n[0], g->quad_lo[0], __builtin_huge_valf(), &t)) {
    for (int c = 0; c < 3; ++c) out[c] = g->env[c];
    return;
  }
  const V3 p = at(o, d, t);
  const V3 n = dp_ground_normal(g);
  const V3 toL = sub(ld3(g->pl[0]), p);
  const float dist = sqrtf(dot(toL, toL));
  const V3 wi = scale(toL, 1.0f / dist);
  float sp[4], ts;
  dp_sphere4(st, sp);
  if (hit_sphere(offset_origin(p, n), wi, sp, dist * 0.9999f, &ts)) {
    out[0] = out[1] = out[2] = 0.0f;
    return;
  }
  dp_shade(g, g->quad_mat[0], p, n, out);
}

// a point of the circle of tangent points seen from `from`, at angle
// fraction frac, and its derivative per radian
__device__ __forceinline__ void dp_tangent_circle(const DpState& st, V3 from, float frac, V3* p, V3* dp) {
  const V3 a = sub(from, st.c);
  const float kk = (st.rho * st.rho) / dot(a, a);
  const V3 cs = mk(st.c.x + a.x * kk, st.c.y + a.y * kk, st.c.z + a.z * kk);
  const float rs = st.rho * sqrtf(1.0f - kk);
  V3 b1, b2;
  basis(unit(a), &b1, &b2);
  float sn, cn;
  sincos_turn(frac, &sn, &cn);
  *p = mk(cs.x + (b1.x * cn + b2.x * sn) * rs, cs.y + (b1.y * cn + b2.y * sn) * rs,
          cs.z + (b1.z * cn + b2.z * sn) * rs);
  *dp = mk((b2.x * cn - b1.x * sn) * rs, (b2.y * cn - b1.y * sn) * rs, (b2.z * cn - b1.z * sn) * rs);
}

// silhouette sample: pixel, radiance step inside - outside, outward normal
// speed per centre axis (pixels per unit), edge length per radian (pixels)
__device__ bool dp_silhouette(const DpState& st, float frac, int* pix, float df[3], float vn[3], float* dl) {
  const SceneHdr* g = st.g;
  const V3 e = ld3(g->eye);
  V3 p, dp;
  dp_tangent_circle(st, e, frac, &p, &dp);
  float px, py;
  V3 jx, jy;
  dp_project(g, p, &px, &py, &jx, &jy);
  if (!(px >= 0.0f && px < (float)g->W && py >= 0.0f && py < (float)g->H)) return false;
  *pix = (int)py * g->W + (int)px;
  const float dx = dot(jx, dp), dy = dot(jy, dp);
  *dl = sqrtf(dx * dx + dy * dy);
  const V3 n = scale(sub(p, st.c), 1.0f / st.rho);
  float fin[3], fout[3];
  dp_shade(g, g->sph_mat[0], p, n, fin);
  const V3 dir = unit(sub(p, e));
  dp_behind(st, e, dir, fout);
  for (int c = 0; c < 3; ++c) df[c] = fin[c] - fout[c];
  const V3 f = ld3(g->fwd), r = ld3(g->right), u = ld3(g->up);
  const V3 pe = sub(p, e);
  const float lam = dot(pe, f);
  const float dlen = sqrtf(dot(pe, pe)) / lam;
  const float q = dot(sub(st.c, e), dir);
  const V3 m = scale(n, -st.rho);
  const float gxx = ((-2.0f * q) / dlen) * (dot(m, r) * (2.0f / (float)g->W));
  const float gyy = ((-2.0f * q) / dlen) * (dot(m, u) * (-2.0f / (float)g->H));
  const float gn = sqrtf(gxx * gxx + gyy * gyy);
  vn[0] = (2.0f * st.rho * n.x) / gn;
  vn[1] = (2.0f * st.rho * n.y) / gn;
  vn[2] = (2.0f * st.rho * n.z) / gn;
  return true;
}

// shadow-boundary sample (see dp_silhouette); the step is the lit radiance
__device__ bool dp_shadow(const DpState& st, float frac, int* pix, float df[3], float vn[3], float* dl) {
  const SceneHdr* g = st.g;
  const V3 e = ld3(g->eye), L = ld3(g->pl[0]);
  V3 t, dt;
  dp_tangent_circle(st, L, frac, &t, &dt);
  const V3 np = dp_ground_normal(g);
  const V3 q0 = ld3(g->quad[0]);
  const V3 tl = sub(t, L);
  const float den = dot(tl, np);
  if (!(den < 0.0f)) return false;
  const float lam = dot(sub(q0, L), np) / den;
  if (!(lam > 1.0f)) return false;
  const V3 gp = at(L, tl, lam);
  // on the ground quad (the same decision as dividing by nn)
  const V3 e1 = ld3(g->quad[0] + 3), e2 = ld3(g->quad[0] + 6), nq = ld3(g->quad_n[0]);
  const float nn = g->quad_n[0][3], lo = g->quad_lo[0];
  const V3 gd = sub(gp, q0);
  const float al = dot(cross(gd, e2), nq), be = dot(cross(e1, gd), nq);
  if (al <= lo || al > nn || be <= lo || be > nn) return false;
  const V3 f = ld3(g->fwd), r = ld3(g->right), u = ld3(g->up);
  const V3 ge = sub(gp, e);
  const float lc = dot(ge, f);
  if (!(lc > 0.0f)) return false;
  float px, py;
  V3 jx, jy;
  dp_project(g, gp, &px, &py, &jx, &jy);
  if (!(px >= 0.0f && px < (float)g->W && py >= 0.0f && py < (float)g->H)) return false;
  const float gdist = sqrtf(dot(ge, ge));
  const V3 wc = scale(ge, 1.0f / gdist);
  float sp[4], tsp;
  dp_sphere4(st, sp);
  if (hit_sphere(e, wc, sp, gdist * 0.9999f, &tsp)) return false;
  *pix = (int)py * g->W + (int)px;
  const float dlam = -lam * (dot(dt, np) / den);
  const V3 dg = mk(dt.x * lam + tl.x * dlam, dt.y * lam + tl.y * dlam, dt.z * lam + tl.z * dlam);
  const float dx = dot(jx, dg), dy = dot(jy, dg);
  *dl = sqrtf(dx * dx + dy * dy);
  dp_shade(g, g->quad_mat[0], gp, np, df);
  const V3 lg = sub(gp, L);
  const float lgd = sqrtf(dot(lg, lg));
  const V3 w = scale(lg, 1.0f / lgd);
  const V3 cl = sub(st.c, L);
  const float qs = dot(cl, w);
  const V3 ms = mk(cl.x - w.x * qs, cl.y - w.y * qs, cl.z - w.z * qs);
  const V3 dd = scale(ge, 1.0f / lc);
  const float dn = dot(dd, np);
  const V3 ddx = scale(r, 2.0f / (float)g->W), ddy = scale(u, -2.0f / (float)g->H);
  const float ax = dot(ddx, np) / dn, ay = dot(ddy, np) / dn;
  const V3 dgx = mk((ddx.x - dd.x * ax) * lc, (ddx.y - dd.y * ax) * lc, (ddx.z - dd.z * ax) * lc);
  const V3 dgy = mk((ddy.x - dd.x * ay) * lc, (ddy.y - dd.y * ay) * lc, (ddy.z - dd.z * ay) * lc);
  const float gxx = ((-2.0f * qs) * dot(ms, dgx)) / lgd;
  const float gyy = ((-2.0f * qs) * dot(ms, dgy)) / lgd;
  const float gn = sqrtf(gxx * gxx + gyy * gyy);
  vn[0] = (2.0f * ms.x) / gn;
  vn[1] = (2.0f * ms.y) / gn;
  vn[2] = (2.0f * ms.z) / gn;
  return true;
}

// interior derivative sample at image point (px, py): df/dc (rgb x axis)
__device__ void dp_interior(const DpState& st, float px, float py, float out[3][3]) {
  const SceneHdr* g = st.g;
  for (int c = 0; c < 3; ++c)
    for (int j = 0; j < 3; ++j) out[c][j] = 0.0f;
  const float sx = 2.0f * (px / (float)g->W) - 1.0f;
  const float sy = 1.0f - 2.0f * (py / (float)g->H);
  const V3 e = ld3(g->eye);
  const V3 d = unit(mk(g->fwd[0] + g->right[0] * sx + g->up[0] * sy, g->fwd[1] + g->right[1] * sx + g->up[1] * sy,
                       g->fwd[2] + g->right[2] * sx + g->up[2] * sy));
  float sp[4], ts, tg;
  dp_sphere4(st, sp);
  if (!hit_sphere(e, d, sp, __builtin_huge_valf(), &ts)) return;
  if (hit_quad(e, d, g->quad[0], g->quad_n[0], g->quad_lo[0], ts, &tg)) return;
  const float rho = st.rho;
  const V3 p = at(e, d, ts);
  const V3 n = scale(sub(p, st.c), 1.0f / rho);
  const V3 v = sub(ld3(g->pl[0]), p);
  const float nv = dot(n, v);
  if (!(nv > 0.0f)) return;
  const float r2 = dot(v, v), rr = sqrtf(r2), r3 = r2 * rr;
  const float dn = dot(d, n);
  const int mat = g->sph_mat[0];
  for (int j = 0; j < 3; ++j) {
    const float nj = j == 0 ? n.x : j == 1 ? n.y : n.z;
    const float dtj = nj / dn;
    const V3 dpj = scale(d, dtj);
    const V3 ej = mk(j == 0 ? 1.0f : 0.0f, j == 1 ? 1.0f : 0.0f, j == 2 ? 1.0f : 0.0f);
    const V3 dnj = scale(sub(dpj, ej), 1.0f / rho);
    const float dnv = dot(dnj, v) - dot(n, dpj);
    const float dvv = -dot(v, dpj);
    const float dg = dnv / r3 - ((3.0f * nv) * dvv) / (r2 * r3);
    for (int ch = 0; ch < 3; ++ch) out[ch][j] = (g->mat_rgb[mat][ch] * kInvPi) * (g->pl[0][3 + ch] * dg);
  }
}

// block sum of d binary64 values in a fixed order (wave butterfly, then waves)
template <int BS>
__device__ __forceinline__ void dp_block_store(double (&acc)[3], int d, double* __restrict__ out) {
  __shared__ double wsum[BS / 64][3];
  for (int j = 0; j < 3; ++j) {
    double v = acc[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < (unsigned)d) {
    double s = 0.0;
    for (int w = 0; w < BS / 64; ++w) s += wsum[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

constexpr int kDpBlock = 256;

// interior term of render k: one thread per pixel, spp derivative samples;
// partial[k][block][j] = sum over the block's pixels of sum_c (I - R)_c mean_s df_c/dc_ax(j)
__global__ __launch_bounds__(kDpBlock) void dp_interior_kernel(const SceneHdr* __restrict__ g,
                                                               const float* __restrict__ X, int d,
                                                               uint32_t k0, uint32_t k1,
                                                               const float* __restrict__ img,
                                                               const float* __restrict__ ref,
                                                               int blocks_per_image,
                                                               double* __restrict__ partial) {
  const int k = blockIdx.x / blocks_per_image, blk = blockIdx.x - k * blocks_per_image;
  const int W = g->W, H = g->H, npix = W * H;
  const int pix = blk * kDpBlock + threadIdx.x;
  const DpState st = dp_state(g, X + (size_t)k * d, d);
  const int pair = k >> 1;
  double acc[3] = {0.0, 0.0, 0.0};
  if (pix < npix) {
    double s[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int smp = 0; smp < g->spp; ++smp) {
      float jx = 0.5f, jy = 0.5f;
      if (!g->pixel_center) {
        const uint4 w = path_words(k0, k1, pix, smp, pair, kTagDiff, 0, 0);
        jx = unit_open(w.x);
        jy = unit_open(w.y);
      }
      float o[3][3];
      dp_interior(st, (float)(pix % W) + jx, (float)(pix / W) + jy, o);
      for (int c = 0; c < 3; ++c)
        for (int j = 0; j < 3; ++j) s[c][j] += (double)o[c][j];
    }
    const float* I = img + ((size_t)k * npix + pix) * 3;
    const float* R = ref + (size_t)pix * 3;
    for (int j = 0; j < d; ++j) {
      const int ax = g->bind_comp[j];
      for (int c = 0; c < 3; ++c) acc[j] += ((double)I[c] - (double)R[c]) * (s[c][ax] / (double)g->spp);
    }
  }
  dp_block_store<kDpBlock>(acc, d, partial + (size_t)blockIdx.x * 3);
}

// edge terms of render k: one thread per edge sample (silhouette samples then
// shadow samples, M each), weighted by the sample pixel's (I - R)
__global__ __launch_bounds__(kDpBlock) void dp_edge_kernel(const SceneHdr* __restrict__ g,
                                                           const float* __restrict__ X, int d,
                                                           uint32_t k0, uint32_t k1,
                                                           const float* __restrict__ img,
                                                           const float* __restrict__ ref, int M,
                                                           int blocks_per_image,
                                                           double* __restrict__ partial) {
  const int k = blockIdx.x / blocks_per_image, blk = blockIdx.x - k * blocks_per_image;
  const int i = blk * kDpBlock + threadIdx.x;
  const DpState st = dp_state(g, X + (size_t)k * d, d);
  double acc[3] = {0.0, 0.0, 0.0};
  if (i < 2 * M) {
    const int edge = i >= M ? 1 : 0, m = i - edge * M;
    const uint4 w = philox10(make_uint4((uint32_t)m, (uint32_t)edge, (uint32_t)(k >> 1),
                                        (uint32_t)kTagEdge << 24), k0, k1);
    const float frac = ((float)m + unit_open(w.x)) / (float)M;
    int pix;
    float df[3], vn[3], dl;
    const bool ok = edge == 0 ? dp_silhouette(st, frac, &pix, df, vn, &dl)
                              : dp_shadow(st, frac, &pix, df, vn, &dl);
    if (ok) {
      const double wgt = (2.0 * 3.14159265358979323846 / (double)M) * (double)dl;
      const size_t npix = (size_t)g->W * g->H;
      const float* I = img + ((size_t)k * npix + pix) * 3;
      const float* R = ref + (size_t)pix * 3;
      for (int j = 0; j < d; ++j) {
        const int ax = g->bind_comp[j];
        for (int c = 0; c < 3; ++c)
          acc[j] += ((double)I[c] - (double)R[c]) * (wgt * (double)df[c] * (double)vn[ax]);
      }
    }
  }
  dp_block_store<kDpBlock>(acc, d, partial + (size_t)blockIdx.x * 3);
}

// g_j = 2/(3HW) (1/N) sum over renders of their interior and edge partials
// (each render's partials in block order), and Q = mean loss
__global__ void dp_combine_kernel(int N, int d, int interior_blocks, int edge_blocks,
                                  const double* __restrict__ pin, const double* __restrict__ pedge,
                                  double inv_den, const double* __restrict__ losses,
                                  double* __restrict__ grad, double* __restrict__ loss) {
  // one wave: lane l sums the block partials l, l + 64, ... of every image
  // (interior, then edge), then a fixed-order butterfly adds the lanes, so the
  // result is reproducible; the images' weights are all 2 / den
  const int l = threadIdx.x;
  for (int j = 0; j < d; ++j) {
    double part = 0.0;
    for (int k = 0; k < N; ++k) {
      for (int b = l; b < interior_blocks; b += 64) part += pin[((size_t)k * interior_blocks + b) * 3 + j];
      for (int b = l; b < edge_blocks; b += 64) part += pedge[((size_t)k * edge_blocks + b) * 3 + j];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    if (l == 0) grad[j] = ((2.0 * inv_den) * part) / (double)N;
  }
  if (l == 0) {
    double s = 0.0;
    for (int k = 0; k < N; ++k) s += losses[k];
    *loss = s / (double)N;
  }
}

// Scratch of the allocation-free estimate (prdpt_grad_estimate_noalloc): one
// fixed array that every device the library runs on holds until the process
// ends.  Host code never passes this name to a kernel (on the host it is a
// stand-in, not a device address); it uses the address noalloc_scratch looked
// up for the device.
static __device__ __align__(256) unsigned char scratch[PRDPT_NOALLOC_SCRATCH_BYTES];

}  // namespace

// ---------------------------------------------------------------------------
// launchers (host)
// ---------------------------------------------------------------------------
hipError_t noalloc_scratch(int device, void** out) {
  static std::mutex mu;
  static void* addr[64] = {};
  if (!out) return hipErrorInvalidValue;
  *out = nullptr;
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *out = addr[device];
  return hipSuccess;
}

int render_tiles(int W, int H, int tile_log2) {
  const int ts = 1 << tile_log2;
  return ((W + ts - 1) / ts) * ((H + ts - 1) / ts);
}

int render_tile_log2(int W, int H, int spp) {
  // 4x4 tiles quadruple the work items of images under 2048 8x8 tiles, which
  // otherwise leave the persistent grid with a few items per work-group and a
  // long tail; 16 samples per pixel still give each item 256 paths
  return (render_tiles(W, H, 3) < 2048 && spp >= 16) ? 2 : 3;
}

hipError_t launch_tau(hipStream_t st, int est, int d, int P, uint64_t seed, const float* sigma,
                      const float* theta, double cd, double sqrt2pi, float* tau, double* c, float* X) {
  const int bs = 64;
  hipLaunchKernelGGL(tau_kernel, dim3((P + bs - 1) / bs), dim3(bs), 0, st, est, d, P,
                     (uint32_t)seed, (uint32_t)(seed >> 32), sigma, theta, cd, sqrt2pi, tau, c, X);
  return hipGetLastError();
}

// Work-groups of a kernel resident at once on a CU of device dev with
// dyn_lds bytes of dynamic LDS: the occupancy calculator's count, capped by
// the count the hardware's 1280-byte LDS allocation units allow (the
// calculator assumes a finer allocation; a persistent grid above the resident
// count leaves work-groups waiting for others to exit).  0 on error.
static int resident_per_cu(int dev, const void* fn, size_t dyn_lds) {
  int per_cu = 0, lds_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, dyn_lds) != hipSuccess)
    return 0;
  hipFuncAttributes fa{};
  if (hipFuncGetAttributes(&fa, fn) == hipSuccess &&
      hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
          hipSuccess && lds_cu > 0) {
    const size_t units = (fa.sharedSizeBytes + dyn_lds + kLdsAllocUnit - 1) / kLdsAllocUnit;
    per_cu = std::min(per_cu, (int)((size_t)lds_cu / (units * kLdsAllocUnit)));
  }
  return std::max(1, per_cu);
}

// resident work-groups of the render kernel on the current device for the
// variant and the dynamic LDS of n_sph spheres (cached)
int render_grid_limit(int rot, int n_sph, int tile_log2) {
  static int cached[64][2][2][PRDPT_MAX_SPHERES + 1];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (n_sph < 0 || n_sph > PRDPT_MAX_SPHERES) return 0;
  rot = rot ? 1 : 0;
  const int small = tile_log2 == 2 ? 1 : 0;
  int& slot = cached[dev][rot][small][n_sph];
  if (slot > 0) return slot;
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const void* fn = rot ? (small ? reinterpret_cast<const void*>(render_loss_kernel<false, true, 2>)
                                : reinterpret_cast<const void*>(render_loss_kernel<false, true, 3>))
                       : (small ? reinterpret_cast<const void*>(render_loss_kernel<false, false, 2>)
                                : reinterpret_cast<const void*>(render_loss_kernel<false, false, 3>));
  const int per_cu = resident_per_cu(dev, fn, (size_t)sphere_lds_bytes(n_sph));
  if (per_cu < 1) return 0;
  slot = n_cu * per_cu;
  return slot;
}

// resident work-groups of the batched render kernel on the current device
// with the dynamic LDS of max_sph spheres (cached)
int batch_grid_limit(int rot, int max_sph) {
  static int cached[64][2][PRDPT_MAX_SPHERES + 1];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (max_sph < 0 || max_sph > PRDPT_MAX_SPHERES) return 0;
  rot = rot ? 1 : 0;
  int& slot = cached[dev][rot][max_sph];
  if (slot > 0) return slot;
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const void* fn = rot ? reinterpret_cast<const void*>(batch_render_kernel<true>)
                       : reinterpret_cast<const void*>(batch_render_kernel<false>);
  const int per_cu = resident_per_cu(dev, fn, (size_t)sphere_lds_bytes(max_sph));
  if (per_cu < 1) return 0;
  slot = n_cu * per_cu;
  return slot;
}

void euler_rotation_host(const float* ang, float* R) { euler_rotation(ang, R); }

// Normal n = edge1 x edge2 of a quad with its squared length, and the unit
// normal with the area, in the operation order of the intersection and the
// shading: cross product, squared length, its sqrt, one reciprocal, three
// products.
// Largest binary32 x whose correctly rounded quotient x / nn is below 0, for
// nn > 0 finite: round(x / nn) < 0 exactly when x < -nn 2^-150 (half the
// smallest subnormal; the tie rounds to -0), so this is minus the smallest
// float above nn 2^-150.  Computed on the bit pattern (no floating-point
// operation, so no dependence on the host's subnormal modes).
float quad_neg_limit_host(float nn) {
  uint32_t b;
  std::memcpy(&b, &nn, 4);
  const uint32_t eb = (b >> 23) & 0xffu, m = b & 0x7fffffu;
  uint32_t y;  // bits of the smallest float above nn 2^-150
  if (eb > 150) {
    y = ((eb - 150) << 23 | m) + 1;  // nn 2^-150 is itself a normal float
  } else if (eb == 0) {
    y = 1;  // subnormal nn: nn 2^-150 is below the smallest subnormal
  } else {
    // nn 2^-150 = (2^23 + m) 2^(eb - 300), in units of the smallest subnormal
    // 2^-149: (2^23 + m) 2^(eb - 151), below one unit shifted out
    const int sh = 151 - (int)eb;
    const uint32_t q = sh >= 32 ? 0u : ((0x800000u | m) >> sh);
    y = q + 1;
  }
  y |= 0x80000000u;
  float out;
  std::memcpy(&out, &y, 4);
  return out;
}

void quad_frame_host(const float* q, float* n, float* nu) {
  const float ax = q[3], ay = q[4], az = q[5], bx = q[6], by = q[7], bz = q[8];
  const float nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
  const float nn = nx * nx + ny * ny + nz * nz;
  const float area = sqrtf(nn);
  const float inv = 1.0f / area;
  n[0] = nx;
  n[1] = ny;
  n[2] = nz;
  n[3] = nn;
  nu[0] = nx * inv;
  nu[1] = ny * inv;
  nu[2] = nz * inv;
  nu[3] = area;
}

hipError_t launch_render(hipStream_t st, const DevScene& sc, int W, int H, int tile_log2,
                         const float* X, int nk,
                         int d, int tag, uint64_t seed, const float* ref, float* img,
                         float* partial, unsigned long long* counters, int* work,
                         const int* order, float* cost, int crn, int rot, int n_sph) {
  const int n_tiles = render_tiles(W, H, tile_log2);
  const long long n_items = (long long)n_tiles * nk;
  if (n_items >= (1ll << 31)) return hipErrorInvalidValue;  // the work counter is an int
  const int limit = render_grid_limit(rot, n_sph, tile_log2);
  if (limit <= 0) return hipErrorInvalidDevice;
  const size_t lds = (size_t)sphere_lds_bytes(n_sph);
  const int blocks = (int)std::min<long long>(n_items, limit);
  hipLaunchKernelGGL(reset_work_kernel, dim3(1), dim3(64), 0, st, work);
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#define PRDPT_RENDER(C, R, L)                                                                      \
  hipLaunchKernelGGL((render_loss_kernel<C, R, L>), dim3(blocks), dim3(kBlock), lds, st, sc, X, d,  \
                     tag, k0, k1, ref, img, partial, counters, n_tiles, (int)n_items, work, order,    \
                     cost, crn)
  // the counting copy reads the tile size from the scene; the timed kernels
  // have it as a constant
  if (counters) {
    if (rot) PRDPT_RENDER(true, true, 0);
    else PRDPT_RENDER(true, false, 0);
  } else if (tile_log2 == 2) {
    if (rot) PRDPT_RENDER(false, true, 2);
    else PRDPT_RENDER(false, false, 2);
  } else {
    if (rot) PRDPT_RENDER(false, true, 3);
    else PRDPT_RENDER(false, false, 3);
  }
#undef PRDPT_RENDER
  return hipGetLastError();
}

hipError_t launch_tile_order(hipStream_t st, const float* cost, int* order, int n_tiles) {
  if (!cost || !order || n_tiles < 1 || n_tiles > kOrderMax) return hipSuccess;
  hipLaunchKernelGGL(tile_order_kernel, dim3(1), dim3(1024), 0, st, cost, order, n_tiles);
  return hipGetLastError();
}

hipError_t launch_losses(hipStream_t st, const float* partial, int n_tiles, int N, int npix,
                         double* losses) {
  hipLaunchKernelGGL(loss_kernel, dim3(N), dim3(64), 0, st, partial, n_tiles, N,
                     1.0 / (3.0 * (double)npix), losses);
  return hipGetLastError();
}

hipError_t launch_combine(hipStream_t st, int rows, int d, int independent, const double* c,
                          const double* L, const double* scale, double* grad, double* loss) {
  hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(64), 0, st, rows, d, independent, c, L, scale,
                     grad, loss);
  return hipGetLastError();
}

// The batch sequence with launch shapes that do not depend on the batch's
// content (totals are read from the device-side meta), so it can be captured
// once in a graph and replayed for every batch.
hipError_t launch_batch(hipStream_t st, const BatchReq* reqs, BatchMeta* meta, int render_blocks,
                        int rot, int max_sph, float* tau, double* c, float* X,
                        float* partial, double* losses, double* grads, double* loss) {
  const size_t lds = (size_t)sphere_lds_bytes(max_sph);
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, st, meta);
  hipLaunchKernelGGL(batch_tau_kernel, dim3(64), dim3(64), 0, st, reqs, meta, tau, c, X);
  if (rot)
    hipLaunchKernelGGL((batch_render_kernel<true>), dim3(render_blocks), dim3(kBlock), lds, st, reqs,
                       meta, X, partial);
  else
    hipLaunchKernelGGL((batch_render_kernel<false>), dim3(render_blocks), dim3(kBlock), lds, st, reqs,
                       meta, X, partial);
  hipLaunchKernelGGL(batch_loss_kernel, dim3(1024), dim3(64), 0, st, reqs, meta, partial, losses);
  hipLaunchKernelGGL(batch_combine_kernel, dim3(256), dim3(64), 0, st, reqs, meta, c, losses,
                     grads, loss);
  return hipGetLastError();
}

int dp_interior_blocks(int W, int H) { return (W * H + kDpBlock - 1) / kDpBlock; }
int dp_edge_blocks(int M) { return (2 * M + kDpBlock - 1) / kDpBlock; }

hipError_t launch_dp(hipStream_t st, const SceneHdr* hdr, int W, int H, const float* X, int N, int d,
                     uint64_t seed, const float* img, const float* ref, int M, double* pin,
                     double* pedge, const double* losses, double* grad, double* loss) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const int bi = dp_interior_blocks(W, H), be = dp_edge_blocks(M);
  hipLaunchKernelGGL(dp_interior_kernel, dim3(N * bi), dim3(kDpBlock), 0, st, hdr, X, d, k0, k1, img,
                     ref, bi, pin);
  hipLaunchKernelGGL(dp_edge_kernel, dim3(N * be), dim3(kDpBlock), 0, st, hdr, X, d, k0, k1, img, ref,
                     M, be, pedge);
  hipLaunchKernelGGL(dp_combine_kernel, dim3(1), dim3(64), 0, st, N, d, bi, be, pin, pedge,
                     1.0 / (3.0 * (double)W * (double)H), losses, grad, loss);
  return hipGetLastError();
}

hipError_t launch_math_selftest(hipStream_t st, unsigned long long* bad) {
  // all 2^32 bit patterns in two halves (the index range of one launch is 32-bit)
  hipLaunchKernelGGL(math_selftest_kernel, dim3(8192), dim3(256), 0, st, 0u, 0x80000000u, bad);
  hipLaunchKernelGGL(math_selftest_kernel, dim3(8192), dim3(256), 0, st, 0x80000000u, 0x80000000u,
                     bad);
  return hipGetLastError();
}

hipError_t launch_copy(hipStream_t st, const void* src, void* dst, size_t n16) {
  const int blocks = 256 * 16;  // 16 work-groups per CU
  hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, st,
                     reinterpret_cast<const float4*>(src), reinterpret_cast<float4*>(dst), n16);
  return hipGetLastError();
}

}  // namespace prdpt
