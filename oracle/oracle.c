/*
 * CPU oracle: plain, slow reference for the plateau-reduced gradient estimator
 * and for the path tracer it wraps as a black box.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it; nothing in the HIP library calls or links it.
 *
 * What it follows (Fischer & Ritschel, "Plateau-reduced Differentiable Path
 * Tracing", CVPR 2023):
 *   - smoothed objective Q = kappa * L (Sec. 3.1, Eq. 6) with a Gaussian kernel
 *     (supplement, kernel definition);
 *   - gradient through the kernel derivative, renderer used as a black box
 *     (Sec. 3.1, Eq. 10; kernel derivative Eq. 11);
 *   - antithetic pairs tau / -tau (Sec. 3.2) and importance sampling of the
 *     positivised kernel derivative, whose magnitude is the inverse-CDF sample
 *     sqrt(-2 sigma^2 ln xi) (Sec. 3.2; supplement, CDF/ICDF derivation);
 *   - image objective: mean squared error against a reference (Sec. 2.1, Eq. 2;
 *     Sec. 4.1 metrics).
 * Readings where the text is ambiguous (missing kernel constant in Alg. 1, the
 * multi-dimensional importance sampler, the dropped kappa weight of Eq. 7) are
 * the ones listed in the design notes; each is marked below where it applies.
 *
 * Precision: per-sample geometry and shading in binary32 (hit decisions are taken
 * in the GPU path's precision), fixed operation order, compiled without
 * floating-point contraction.  All sums are binary64.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
#define INV_PI_F 0.318309886183790671538f

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, written from Salmon, Moraes, Dror & Shaw, "Parallel random  */
/* numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two 32x32->64          */
/* multiplications with the Weyl key schedule.                                */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void seed_key(uint64_t seed, uint32_t key[2]) {
  key[0] = (uint32_t)seed;
  key[1] = (uint32_t)(seed >> 32);
}

/* Uniform on the open interval (0,1): top 23 bits plus one half, times 2^-23.
 * Every value is exact in binary32 and lies in [2^-24, 1 - 2^-24]. */
float orc_u01(uint32_t x) { return ((float)(x >> 9) + 0.5f) * 1.1920928955078125e-07f; }

/* Natural logarithm for positive normal binary32 input, from IEEE basic
 * operations only: x = m 2^e with m in [sqrt(1/2), sqrt(2)],
 * ln m = 2 atanh(s), s = (m-1)/(m+1), atanh by its odd power series through s^11,
 * and e ln 2 split into a short high part and a low correction. */
float orc_ln(float x) {
  uint32_t b;
  memcpy(&b, &x, 4);
  int e = (int)((b >> 23) & 0xffu) - 127;
  uint32_t mb = (b & 0x007fffffu) | 0x3f800000u;
  float m;
  memcpy(&m, &mb, 4);
  if (m > 1.41421356f) {
    m = m * 0.5f;
    e = e + 1;
  }
  float s = (m - 1.0f) / (m + 1.0f);
  float s2 = s * s;
  float p = 1.0f / 11.0f;
  p = 1.0f / 9.0f + s2 * p;
  p = 1.0f / 7.0f + s2 * p;
  p = 1.0f / 5.0f + s2 * p;
  p = 1.0f / 3.0f + s2 * p;
  float at = s + s * (s2 * p);
  float lm = at + at;
  float fe = (float)e;
  return fe * 0.693145751953125f + (lm + fe * 1.42860677e-06f);
}

/* sin(2 pi u) and cos(2 pi u) for u in [0, 1): exact reduction to a quarter
 * turn index q and a remainder r in [-1/8, 1/8], then the Taylor series of sin
 * (through x^9) and cos (through x^10) at x = 2 pi r, then the quarter-turn
 * rotation. */
void orc_sincos_2pi(float u, float* s_out, float* c_out) {
  float u4 = u * 4.0f;
  int q = (int)u4;
  float r = u - (float)q * 0.25f;
  if (r > 0.125f) {
    r = r - 0.25f;
    q = q + 1;
  }
  float x = r * 6.28318530717958647692f;
  float x2 = x * x;
  float ps = -1.0f / 5040.0f + x2 * (1.0f / 362880.0f);
  ps = 1.0f / 120.0f + x2 * ps;
  ps = -1.0f / 6.0f + x2 * ps;
  float sn = x + x * (x2 * ps);
  float pc = 1.0f / 40320.0f + x2 * (-1.0f / 3628800.0f);
  pc = -1.0f / 720.0f + x2 * pc;
  pc = 1.0f / 24.0f + x2 * pc;
  pc = -0.5f + x2 * pc;
  float cs = 1.0f + x2 * pc;
  switch (q & 3) {
    case 0: *s_out = sn; *c_out = cs; break;
    case 1: *s_out = cs; *c_out = -sn; break;
    case 2: *s_out = -sn; *c_out = -cs; break;
    default: *s_out = -cs; *c_out = sn; break;
  }
}

/* Mean of the chi distribution with d degrees of freedom,
 * sqrt(2) Gamma((d+1)/2) / Gamma(d/2), by C_1 = sqrt(2/pi), C_{k+1} = k / C_k. */
double orc_chi_mean(int d) {
  double c = sqrt(2.0 / ORC_PI);
  for (int k = 1; k < d; ++k) c = (double)k / c;
  return c;
}

/* ------------------------------------------------------------------------- */
/* Perturbation draw (Sec. 3.2).  Words of the TAU stream for pair p are      */
/* Philox(counter = (p, block, 0, TAU<<24)), consumed four per block, in order.*/
/* ------------------------------------------------------------------------- */
typedef struct {
  uint32_t key[2];
  uint32_t pair, block;
  uint32_t w[4];
  int used;
  int strata;  /* > 0: the draw's first uniform lies in stratum `pair` of this many */
} tau_stream;

static uint32_t tau_word(tau_stream* st) {
  if (st->used == 4) {
    uint32_t ctr[4] = {st->pair, st->block, 0u, (uint32_t)ORC_TAG_TAU << 24};
    orc_philox4x32_10(ctr, st->key, st->w);
    st->block++;
    st->used = 0;
  }
  return st->w[st->used++];
}

/* the next uniform of the draw; with strata, the first one is (i + u) / P for
 * draw i of P (binary32, kept below 1) */
static float tau_uniform(tau_stream* st) {
  float u = orc_u01(tau_word(st));
  if (st->strata > 0) {
    u = fminf(((float)st->pair + u) / (float)st->strata, 0x1.fffffep-1f);
    st->strata = 0;
  }
  return u;
}

/* one Box-Muller pair of standard normals from two uniforms */
static void normal_pair(tau_stream* st, float* z0, float* z1) {
  float u1 = tau_uniform(st);
  float u2 = tau_uniform(st);
  float rad = sqrtf(-2.0f * orc_ln(u1));
  float sn, cs;
  orc_sincos_2pi(u2, &sn, &cs);
  *z0 = rad * cs;
  *z1 = rad * sn;
}

int orc_draw_tau(int mode, int d, int P, uint64_t seed, const float* sigma, float* tau,
                 double* c) {
  if (d < 1 || d > ORC_MAX_PARAMS || P < 1) return -1;
  /* independent draws: the same samplers; the weight is the single-sample score
   * weight (its expectation over the draw is the gradient by itself), written
   * below directly: v_j / sigma_j, C_d u_j / sigma_j, s_j 2 / (sigma_j sqrt(2 pi)) */
  const int indep = (mode & ORC_EST_INDEPENDENT) != 0;
  const int strat = (mode & ORC_EST_STRATIFIED) != 0;
  if (strat && !indep) return -1;  /* strata replace the antithetic partner */
  mode &= ~(ORC_EST_INDEPENDENT | ORC_EST_STRATIFIED);
  double cd = orc_chi_mean(d);
  const double sqrt2pi = sqrt(2.0 * ORC_PI);
  float v[ORC_MAX_PARAMS], z[ORC_MAX_PARAMS];
  for (int p = 0; p < P; ++p) {
    tau_stream st;
    seed_key(seed, st.key);
    st.pair = (uint32_t)p;
    st.block = 0;
    st.used = 4;
    st.strata = strat ? P : 0;
    if (mode == ORC_EST_GAUSS) {
      /* tau ~ kappa: v standard normal; pair weight v_j / (2 sigma_j) is the
       * antithetic average of the score (tau_j / sigma_j^2) (Eq. 10, 11). */
      for (int j = 0; j < d; j += 2) {
        float z0, z1;
        normal_pair(&st, &z0, &z1);
        v[j] = z0;
        if (j + 1 < d) v[j + 1] = z1;
      }
      for (int j = 0; j < d; ++j) {
        tau[p * d + j] = sigma[j] * v[j];
        c[p * d + j] = indep ? (double)v[j] / (double)sigma[j]
                             : (double)v[j] / (2.0 * (double)sigma[j]);
      }
    } else if (mode == ORC_EST_IS) {
      /* importance sampling of the kernel derivative: radius rho ~ chi_{d+1}
       * (for d = 1 this is the inverse CDF sqrt(-2 ln xi) of Sec. 3.2), direction
       * uniform; pair weight C_d u_j / (2 sigma_j). */
      int m = (d + 1) / 2;
      float acc = 0.0f;
      for (int i = 0; i < m; ++i) acc = acc + orc_ln(tau_uniform(&st));
      float rho2 = -2.0f * acc;
      if ((d + 1) & 1) {
        float z0, z1;
        normal_pair(&st, &z0, &z1);
        rho2 = rho2 + z0 * z0;
      }
      for (int j = 0; j < d; j += 2) {
        float z0, z1;
        normal_pair(&st, &z0, &z1);
        z[j] = z0;
        if (j + 1 < d) z[j + 1] = z1;
      }
      float n2 = 0.0f;
      for (int j = 0; j < d; ++j) n2 = n2 + z[j] * z[j];
      float nrm = sqrtf(n2);
      float rho = sqrtf(rho2);
      for (int j = 0; j < d; ++j) {
        float uj = z[j] / nrm;
        tau[p * d + j] = sigma[j] * (rho * uj);
        c[p * d + j] = indep ? cd * (double)uj / (double)sigma[j]
                             : cd * (double)uj / (2.0 * (double)sigma[j]);
      }
    } else if (mode == ORC_EST_IS_PERDIM) {
      /* literal per-dimension reading: independent two-sided Rayleigh per axis;
       * the signs come after the radii, one word per 32 axes (bit j mod 32) */
      for (int j = 0; j < d; ++j) v[j] = sqrtf(-2.0f * orc_ln(tau_uniform(&st)));
      uint32_t bits = 0;
      for (int j = 0; j < d; ++j) {
        if (j % 32 == 0) bits = tau_word(&st);
        float sgn = ((bits >> (j % 32)) & 1u) ? -1.0f : 1.0f;
        tau[p * d + j] = sigma[j] * (sgn * v[j]);
        c[p * d + j] = indep ? 2.0 * (double)sgn / ((double)sigma[j] * sqrt2pi)
                             : (double)sgn / ((double)sigma[j] * sqrt2pi);
      }
    } else {
      return -1;
    }
  }
  return 0;
}

/* Eq. 10 with antithetic pairs: g_j = (1/P) sum_p c_pj (L(theta+tau_p) - L(theta-tau_p)) */
void orc_combine(int P, int d, const double* c, const double* L, double* g, double* q) {
  for (int j = 0; j < d; ++j) {
    double acc = 0.0;
    for (int p = 0; p < P; ++p) acc += c[p * d + j] * (L[2 * p] - L[2 * p + 1]);
    g[j] = acc / (double)P;
  }
  if (q) {
    double s = 0.0;
    for (int k = 0; k < 2 * P; ++k) s += L[k];
    *q = s / (double)(2 * P);
  }
}

/* Without antithetic partners: g_j = (1/N) sum_i c_ij L(theta+tau_i) (Eq. 10
 * as a plain Monte Carlo mean of score-weighted losses), Q = mean L */
void orc_combine_independent(int N, int d, const double* c, const double* L, double* g,
                             double* q) {
  for (int j = 0; j < d; ++j) {
    double acc = 0.0;
    for (int i = 0; i < N; ++i) acc += c[i * d + j] * L[i];
    g[j] = acc / (double)N;
  }
  if (q) {
    double s = 0.0;
    for (int i = 0; i < N; ++i) s += L[i];
    *q = s / (double)N;
  }
}

/* ------------------------------------------------------------------------- */
/* vector helpers (binary32, fixed evaluation order)                          */
/* ------------------------------------------------------------------------- */
typedef struct { float x, y, z; } v3;
static inline v3 V(float x, float y, float z) { v3 r = {x, y, z}; return r; }
static inline v3 vsub(v3 a, v3 b) { return V(a.x - b.x, a.y - b.y, a.z - b.z); }
static inline v3 vneg(v3 a) { return V(-a.x, -a.y, -a.z); }
static inline v3 vscale(v3 a, float s) { return V(a.x * s, a.y * s, a.z * s); }
static inline float vdot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline v3 vcross(v3 a, v3 b) {
  return V(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static inline v3 vnorm(v3 a) {
  float len = sqrtf(vdot(a, a));
  float inv = 1.0f / len;
  return vscale(a, inv);
}
static inline v3 vld(const float* p) { return V(p[0], p[1], p[2]); }
/* point along a ray: o + t d */
static inline v3 vray(v3 o, v3 d, float t) { return V(o.x + d.x * t, o.y + d.y * t, o.z + d.z * t); }

/* ------------------------------------------------------------------------- */
/* scene and a simple median-split BVH over each mesh's triangles             */
/* ------------------------------------------------------------------------- */
typedef struct {
  double lo[3], hi[3];
  int32_t left, right, first, count;
} bnode;

typedef struct {
  int n_nodes, cap;
  bnode* nodes;
  int32_t* idx;  /* local triangle indices, leaf ranges refer into this */
} bvh_t;

struct orc_scene {
  float eye[3], fwd[3], right[3], up[3], env[3];
  int W, H, spp, B, pixel_center;
  int n_mat, n_sph, n_quad, n_mesh, n_tri, n_pl, n_param;
  int32_t* mat_type; float* mat_rgb; float* mat_ior;
  float* sph; int32_t* sph_mat;
  float* quad; int32_t* quad_mat;
  int32_t* mesh_off; int32_t* mesh_mat; float* mesh_xlate; float* mesh_rot;
  float* tri;
  float* pl;
  int32_t* binding;
  bvh_t* bvh;
  int brute;
};

typedef struct {
  double key;
  int32_t idx;
} keyed;

static int cmp_keyed(const void* a, const void* b) {
  double ka = ((const keyed*)a)->key, kb = ((const keyed*)b)->key;
  if (ka < kb) return -1;
  if (ka > kb) return 1;
  return ((const keyed*)a)->idx - ((const keyed*)b)->idx;
}

static int bvh_push(bvh_t* b) {
  if (b->n_nodes == b->cap) {
    b->cap = b->cap ? b->cap * 2 : 64;
    b->nodes = (bnode*)realloc(b->nodes, sizeof(bnode) * (size_t)b->cap);
  }
  return b->n_nodes++;
}

static int bvh_build_rec(bvh_t* b, const float* tri, int32_t* idx, int n, int first,
                         keyed* scratch) {
  int ni = bvh_push(b);
  double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
  double clo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, chi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
  for (int i = 0; i < n; ++i) {
    const float* t = tri + 9 * (size_t)idx[i];
    for (int a = 0; a < 3; ++a) {
      double c = 0.0;
      for (int k = 0; k < 3; ++k) {
        double x = t[3 * k + a];
        if (x < lo[a]) lo[a] = x;
        if (x > hi[a]) hi[a] = x;
        c += x;
      }
      c /= 3.0;
      if (c < clo[a]) clo[a] = c;
      if (c > chi[a]) chi[a] = c;
    }
  }
  /* pad so that binary32 hit points of triangles inside are always inside */
  double mag = 1.0;
  for (int a = 0; a < 3; ++a) {
    if (fabs(lo[a]) > mag) mag = fabs(lo[a]);
    if (fabs(hi[a]) > mag) mag = fabs(hi[a]);
  }
  for (int a = 0; a < 3; ++a) {
    b->nodes[ni].lo[a] = lo[a] - 1e-4 * mag;
    b->nodes[ni].hi[a] = hi[a] + 1e-4 * mag;
  }
  if (n <= 4) {
    b->nodes[ni].left = b->nodes[ni].right = -1;
    b->nodes[ni].first = first;
    b->nodes[ni].count = n;
    return ni;
  }
  int axis = 0;
  for (int a = 1; a < 3; ++a)
    if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
  for (int i = 0; i < n; ++i) {
    const float* t = tri + 9 * (size_t)idx[i];
    scratch[i].key = ((double)t[axis] + (double)t[3 + axis] + (double)t[6 + axis]) / 3.0;
    scratch[i].idx = idx[i];
  }
  qsort(scratch, (size_t)n, sizeof(keyed), cmp_keyed);
  for (int i = 0; i < n; ++i) idx[i] = scratch[i].idx;
  int h = n / 2;
  int l = bvh_build_rec(b, tri, idx, h, first, scratch);
  int r = bvh_build_rec(b, tri, idx + h, n - h, first + h, scratch);
  b->nodes[ni].left = l;
  b->nodes[ni].right = r;
  b->nodes[ni].first = 0;
  b->nodes[ni].count = 0;
  return ni;
}

#define DUP(dst, src, n, T)                                   \
  do {                                                        \
    size_t bytes_ = sizeof(T) * (size_t)((n) > 0 ? (n) : 1);  \
    dst = (T*)malloc(bytes_);                                 \
    if ((n) > 0) memcpy(dst, src, sizeof(T) * (size_t)(n));   \
  } while (0)

orc_scene* orc_scene_new(const orc_scene_in* in) {
  orc_scene* s = (orc_scene*)calloc(1, sizeof(orc_scene));
  memcpy(s->eye, in->eye, 12);
  memcpy(s->fwd, in->fwd, 12);
  memcpy(s->right, in->right, 12);
  memcpy(s->up, in->up, 12);
  memcpy(s->env, in->env, 12);
  s->W = in->width; s->H = in->height; s->spp = in->spp; s->B = in->max_bounces;
  s->pixel_center = in->pixel_center;
  s->n_mat = in->n_mat; s->n_sph = in->n_sph; s->n_quad = in->n_quad;
  s->n_mesh = in->n_mesh; s->n_tri = in->n_tri; s->n_pl = in->n_plight;
  s->n_param = in->n_param;
  DUP(s->mat_type, in->mat_type, in->n_mat, int32_t);
  DUP(s->mat_rgb, in->mat_rgb, 3 * in->n_mat, float);
  DUP(s->mat_ior, in->mat_ior, in->n_mat, float);
  DUP(s->sph, in->sph, 4 * in->n_sph, float);
  DUP(s->sph_mat, in->sph_mat, in->n_sph, int32_t);
  DUP(s->quad, in->quad, 9 * in->n_quad, float);
  DUP(s->quad_mat, in->quad_mat, in->n_quad, int32_t);
  DUP(s->mesh_off, in->mesh_off, in->n_mesh + 1, int32_t);
  DUP(s->mesh_mat, in->mesh_mat, in->n_mesh, int32_t);
  DUP(s->mesh_xlate, in->mesh_xlate, 3 * in->n_mesh, float);
  s->mesh_rot = (float*)calloc((size_t)(in->n_mesh > 0 ? 3 * in->n_mesh : 1), sizeof(float));
  if (in->mesh_rot) memcpy(s->mesh_rot, in->mesh_rot, sizeof(float) * 3 * (size_t)in->n_mesh);
  DUP(s->tri, in->tri, 9 * in->n_tri, float);
  DUP(s->pl, in->plight, 6 * in->n_plight, float);
  DUP(s->binding, in->binding, 3 * in->n_param, int32_t);
  s->bvh = (bvh_t*)calloc((size_t)(s->n_mesh > 0 ? s->n_mesh : 1), sizeof(bvh_t));
  for (int m = 0; m < s->n_mesh; ++m) {
    int first = s->mesh_off[m], n = s->mesh_off[m + 1] - first;
    bvh_t* b = &s->bvh[m];
    b->idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) b->idx[i] = first + i;
    if (n > 0) {
      keyed* scratch = (keyed*)malloc(sizeof(keyed) * (size_t)n);
      bvh_build_rec(b, s->tri, b->idx, n, 0, scratch);
      free(scratch);
    }
  }
  return s;
}

void orc_scene_free(orc_scene* s) {
  if (!s) return;
  for (int m = 0; m < s->n_mesh; ++m) {
    free(s->bvh[m].nodes);
    free(s->bvh[m].idx);
  }
  free(s->bvh);
  free(s->mat_type); free(s->mat_rgb); free(s->mat_ior);
  free(s->sph); free(s->sph_mat); free(s->quad); free(s->quad_mat);
  free(s->mesh_off); free(s->mesh_mat); free(s->mesh_xlate); free(s->mesh_rot);
  free(s->tri); free(s->pl); free(s->binding);
  free(s);
}

void orc_set_brute_force(orc_scene* s, int on) { s->brute = on; }

/* Scene state at one parameter vector X: each bound field is base + X_j. */
typedef struct {
  float* sph;
  float* quad;
  float* xlate;
  float* pl;
  float* rgb;   /* material colours */
  float* ang;   /* mesh rotation angles */
  float* rot;   /* [n_mesh][3][3] row-major rotation of each mesh (binary32) */
} kstate;

/* Rotation by the angles (a, b, c) about the fixed x, y and z axes, applied in
 * that order: R = Rz(c) Ry(b) Rx(a), formed as a product of the three axis
 * rotations in binary64 and rounded to binary32. */
static void euler_matrix(const float ang[3], float R[9]) {
  double A[3][3][3];
  for (int ax = 0; ax < 3; ++ax) {
    const double cs = cos((double)ang[ax]), sn = sin((double)ang[ax]);
    const int u = (ax + 1) % 3, w = (ax + 2) % 3;  /* the plane the axis rotates */
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) A[ax][r][c] = r == c ? 1.0 : 0.0;
    A[ax][u][u] = cs; A[ax][u][w] = -sn;
    A[ax][w][u] = sn; A[ax][w][w] = cs;
  }
  double T[3][3], M[3][3];
  for (int r = 0; r < 3; ++r)       /* T = Ry Rx */
    for (int c = 0; c < 3; ++c) {
      T[r][c] = 0.0;
      for (int i = 0; i < 3; ++i) T[r][c] += A[1][r][i] * A[0][i][c];
    }
  for (int r = 0; r < 3; ++r)       /* M = Rz T */
    for (int c = 0; c < 3; ++c) {
      M[r][c] = 0.0;
      for (int i = 0; i < 3; ++i) M[r][c] += A[2][r][i] * T[i][c];
    }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) R[3 * r + c] = (float)M[r][c];
}

static void kstate_init(const orc_scene* s, const float* X, kstate* k) {
  DUP(k->sph, s->sph, 4 * s->n_sph, float);
  DUP(k->quad, s->quad, 9 * s->n_quad, float);
  DUP(k->xlate, s->mesh_xlate, 3 * s->n_mesh, float);
  DUP(k->pl, s->pl, 6 * s->n_pl, float);
  DUP(k->rgb, s->mat_rgb, 3 * s->n_mat, float);
  DUP(k->ang, s->mesh_rot, 3 * s->n_mesh, float);
  for (int j = 0; j < s->n_param; ++j) {
    int kind = s->binding[3 * j], i = s->binding[3 * j + 1], c = s->binding[3 * j + 2];
    if (kind == ORC_BIND_SPHERE) k->sph[4 * i + c] = s->sph[4 * i + c] + X[j];
    else if (kind == ORC_BIND_QUAD) k->quad[9 * i + c] = s->quad[9 * i + c] + X[j];
    else if (kind == ORC_BIND_MESH) k->xlate[3 * i + c] = s->mesh_xlate[3 * i + c] + X[j];
    else if (kind == ORC_BIND_PLIGHT) k->pl[6 * i + c] = s->pl[6 * i + c] + X[j];
    else if (kind == ORC_BIND_ALBEDO) k->rgb[3 * i + c] = s->mat_rgb[3 * i + c] + X[j];
    else if (kind == ORC_BIND_MESH_ROT) k->ang[3 * i + c] = s->mesh_rot[3 * i + c] + X[j];
  }
  k->rot = (float*)malloc(sizeof(float) * 9 * (size_t)(s->n_mesh > 0 ? s->n_mesh : 1));
  for (int m = 0; m < s->n_mesh; ++m) euler_matrix(k->ang + 3 * m, k->rot + 9 * m);
}

static void kstate_free(kstate* k) {
  free(k->sph); free(k->quad); free(k->xlate); free(k->pl); free(k->rgb);
  free(k->ang); free(k->rot);
}

/* ------------------------------------------------------------------------- */
/* primitive tests (binary32, t > 0 and t < tmax)                             */
/* ------------------------------------------------------------------------- */
static int sphere_test(v3 o, v3 d, const float* sp, float tmax, float* tout) {
  v3 c = vld(sp);
  float r = sp[3];
  v3 oc = vsub(o, c);
  float a = vdot(d, d);
  float b = vdot(oc, d);
  float cc = vdot(oc, oc) - r * r;
  float disc = b * b - a * cc;
  if (disc < 0.0f) return 0;
  float sq = sqrtf(disc);
  float q = (b >= 0.0f) ? -(b + sq) : -(b - sq);
  if (q == 0.0f) return 0;
  float t0 = q / a, t1 = cc / q;
  float tn = t0 < t1 ? t0 : t1;
  float tf = t0 < t1 ? t1 : t0;
  float t = tn > 0.0f ? tn : tf;
  if (!(t > 0.0f && t < tmax)) return 0;
  *tout = t;
  return 1;
}

static int quad_test(v3 o, v3 d, const float* qd, float tmax, float* tout) {
  v3 qo = vld(qd), e1 = vld(qd + 3), e2 = vld(qd + 6);
  v3 n = vcross(e1, e2);
  float denom = vdot(n, d);
  if (denom == 0.0f) return 0;
  float t = vdot(n, vsub(qo, o)) / denom;
  if (!(t > 0.0f && t < tmax)) return 0;
  v3 p = vray(o, d, t);
  v3 pd = vsub(p, qo);
  float nn = vdot(n, n);
  float al = vdot(vcross(pd, e2), n) / nn;
  if (al < 0.0f || al > 1.0f) return 0;
  float be = vdot(vcross(e1, pd), n) / nn;
  if (be < 0.0f || be > 1.0f) return 0;
  *tout = t;
  return 1;
}

/* Moeller-Trumbore with edges e1 = v1 - v0, e2 = v2 - v0 */
static int tri_test(v3 o, v3 d, const float* tv, float tmax, float* tout) {
  v3 v0 = vld(tv), v1 = vld(tv + 3), v2 = vld(tv + 6);
  v3 e1 = vsub(v1, v0), e2 = vsub(v2, v0);
  v3 pv = vcross(d, e2);
  float det = vdot(e1, pv);
  if (det == 0.0f) return 0;
  float inv = 1.0f / det;
  v3 tv0 = vsub(o, v0);
  float u = vdot(tv0, pv) * inv;
  if (u < 0.0f || u > 1.0f) return 0;
  v3 qv = vcross(tv0, e1);
  float v = vdot(d, qv) * inv;
  if (v < 0.0f || u + v > 1.0f) return 0;
  float t = vdot(e2, qv) * inv;
  if (!(t > 0.0f && t < tmax)) return 0;
  *tout = t;
  return 1;
}

typedef struct {
  float t;
  int32_t id;
} hitrec;

/* closest hit: smallest t, ties to the smaller primitive id */
static inline void consider(hitrec* h, float t, int32_t id) {
  if (t < h->t || (t == h->t && id < h->id)) {
    h->t = t;
    h->id = id;
  }
}

static int box_hit(const bnode* nd, const double o[3], const double d[3], double tlim) {
  double t0 = 0.0, t1 = tlim;
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0.0) {
      if (o[a] < nd->lo[a] || o[a] > nd->hi[a]) return 0;
      continue;
    }
    double ta = (nd->lo[a] - o[a]) / d[a], tb = (nd->hi[a] - o[a]) / d[a];
    if (ta > tb) { double x = ta; ta = tb; tb = x; }
    if (ta > t0) t0 = ta;
    if (tb < t1) t1 = tb;
    if (t0 > t1) return 0;
  }
  return 1;
}

static void mesh_hit(const orc_scene* s, int m, v3 o, v3 d, float tmax, int base_id, hitrec* h) {
  const bvh_t* b = &s->bvh[m];
  int first = s->mesh_off[m], n = s->mesh_off[m + 1] - first;
  if (n <= 0) return;
  if (s->brute) {
    for (int i = 0; i < n; ++i) {
      float t;
      if (tri_test(o, d, s->tri + 9 * (size_t)(first + i), tmax, &t)) consider(h, t, base_id + first + i);
    }
    return;
  }
  double od[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
  int stack[128];
  int sp = 0;
  stack[sp++] = 0;
  while (sp > 0) {
    const bnode* nd = &b->nodes[stack[--sp]];
    double tlim = (double)(h->t < tmax ? h->t : tmax);
    if (!box_hit(nd, od, dd, tlim)) continue;
    if (nd->count > 0) {
      for (int i = 0; i < nd->count; ++i) {
        int ti = b->idx[nd->first + i];
        float t;
        if (tri_test(o, d, s->tri + 9 * (size_t)ti, tmax, &t)) consider(h, t, base_id + ti);
      }
    } else {
      stack[sp++] = nd->left;
      stack[sp++] = nd->right;
    }
  }
}

/* closest primitive along (o, d) with t in (0, tmax); occluders_only skips lights */
static void closest(const orc_scene* s, const kstate* k, v3 o, v3 d, float tmax,
                    int occluders_only, hitrec* h) {
  h->t = INFINITY;
  h->id = -1;
  for (int i = 0; i < s->n_sph; ++i) {
    float t;
    if (sphere_test(o, d, k->sph + 4 * i, tmax, &t)) consider(h, t, i);
  }
  for (int i = 0; i < s->n_quad; ++i) {
    if (occluders_only && s->mat_type[s->quad_mat[i]] == ORC_EMISSIVE) continue;
    float t;
    if (quad_test(o, d, k->quad + 9 * i, tmax, &t)) consider(h, t, s->n_sph + i);
  }
  int tri_base = s->n_sph + s->n_quad;
  for (int m = 0; m < s->n_mesh; ++m) {
    /* a mesh is an instance: the ray goes into the mesh's own frame by the
     * inverse transform, R^T (o - translation) and R^T d (R orthonormal keeps
     * the ray parameter t of a hit) */
    const float* R = k->rot + 9 * m;
    v3 q = V(o.x - k->xlate[3 * m], o.y - k->xlate[3 * m + 1], o.z - k->xlate[3 * m + 2]);
    v3 om = V(R[0] * q.x + R[3] * q.y + R[6] * q.z, R[1] * q.x + R[4] * q.y + R[7] * q.z,
              R[2] * q.x + R[5] * q.y + R[8] * q.z);
    v3 dm = V(R[0] * d.x + R[3] * d.y + R[6] * d.z, R[1] * d.x + R[4] * d.y + R[7] * d.z,
              R[2] * d.x + R[5] * d.y + R[8] * d.z);
    mesh_hit(s, m, om, dm, tmax, tri_base, h);
  }
}

void orc_trace(const orc_scene* s, const float* X, int n, const float* o, const float* d,
               float* t_out, int32_t* id_out) {
  kstate k;
  kstate_init(s, X, &k);
  for (int i = 0; i < n; ++i) {
    hitrec h;
    closest(s, &k, vld(o + 3 * i), vld(d + 3 * i), INFINITY, 0, &h);
    t_out[i] = h.t;
    id_out[i] = h.id;
  }
  kstate_free(&k);
}

/* material and unit geometric normal (not oriented) of a primitive at point p */
static void prim_info(const orc_scene* s, const kstate* k, int id, v3 p, int* mat, v3* ng) {
  if (id < s->n_sph) {
    *mat = s->sph_mat[id];
    *ng = vnorm(vsub(p, vld(k->sph + 4 * id)));
    return;
  }
  id -= s->n_sph;
  if (id < s->n_quad) {
    *mat = s->quad_mat[id];
    *ng = vnorm(vcross(vld(k->quad + 9 * id + 3), vld(k->quad + 9 * id + 6)));
    return;
  }
  id -= s->n_quad;
  int m = 0;
  while (s->mesh_off[m + 1] <= id) ++m;
  *mat = s->mesh_mat[m];
  const float* tv = s->tri + 9 * (size_t)id;
  v3 v0 = vld(tv);
  v3 nl = vcross(vsub(vld(tv + 3), v0), vsub(vld(tv + 6), v0));  /* mesh frame */
  const float* R = k->rot + 9 * m;
  *ng = vnorm(V(R[0] * nl.x + R[1] * nl.y + R[2] * nl.z, R[3] * nl.x + R[4] * nl.y + R[5] * nl.z,
                R[6] * nl.x + R[7] * nl.y + R[8] * nl.z));
}

/* origin moved off the surface along n by 1e-4 max(1, |p|_inf) */
static v3 spawn(v3 p, v3 n) {
  float m = fmaxf(fabsf(p.x), fmaxf(fabsf(p.y), fabsf(p.z)));
  float eps = 1e-4f * fmaxf(1.0f, m);
  return V(p.x + n.x * eps, p.y + n.y * eps, p.z + n.z * eps);
}

/* orthonormal basis around unit n (Duff et al., JCGT 6(1), 2017) */
static void onb(v3 n, v3* b1, v3* b2) {
  float sign = copysignf(1.0f, n.z);
  float a = -1.0f / (sign + n.z);
  float b = n.x * n.y * a;
  *b1 = V(1.0f + sign * n.x * n.x * a, sign * b, -sign * n.x);
  *b2 = V(b, sign + n.y * n.y * a, -n.y);
}

float orc_fresnel(float cosi, float ei, float et) {
  float eta = ei / et;
  float sin2t = (eta * eta) * (1.0f - cosi * cosi);
  if (sin2t >= 1.0f) return 1.0f;
  float cost = sqrtf(1.0f - sin2t);
  float rs = (ei * cosi - et * cost) / (ei * cosi + et * cost);
  float rp = (et * cosi - ei * cost) / (et * cosi + ei * cost);
  return 0.5f * (rs * rs + rp * rp);
}

/* Cosine-weighted direction about the unit normal n (density cos(theta)/pi on
 * the hemisphere of n): a uniform point of the unit disc, radius sqrt(u1) and
 * angle 2 pi u2, lifted to the hemisphere, z = sqrt(1 - u1), expressed in the
 * orthonormal basis of n and normalised. */
void orc_cosine_direction(const float nin[3], float u1, float u2, float out[3]) {
  v3 n = V(nin[0], nin[1], nin[2]);
  float r = sqrtf(u1);
  float sn, cs;
  orc_sincos_2pi(u2, &sn, &cs);
  float lx = r * cs, ly = r * sn, lz = sqrtf(1.0f - u1);
  v3 b1, b2;
  onb(n, &b1, &b2);
  v3 nd = vnorm(V(b1.x * lx + b2.x * ly + n.x * lz, b1.y * lx + b2.y * ly + n.y * lz,
                  b1.z * lx + b2.z * ly + n.z * lz));
  out[0] = nd.x; out[1] = nd.y; out[2] = nd.z;
}

/* Smooth dielectric interface of index ior (outside index 1): the ray of unit
 * direction d meets a surface with unit geometric normal ng (pointing out of
 * the body).  The normal is turned against d and the indices swapped when the
 * ray leaves the body.  With probability F (exact unpolarised Fresnel; F = 1
 * under total internal reflection), chosen by u < F, the ray is mirrored and
 * the new origin goes to the incident side; otherwise it is refracted by
 * Snell's law, eta_i sin(theta_i) = eta_t sin(theta_t), written in vector form
 * t = eta d + (eta cos_i - cos_t) n with eta = eta_i / eta_t, and the origin
 * goes to the far side.  out: the unit new direction; side: the unit normal
 * of the side the new origin is offset to. */
void orc_dielectric_scatter(const float din[3], const float ngin[3], float ior, float u,
                            float out[3], float side_out[3]) {
  v3 d = V(din[0], din[1], din[2]);
  v3 n = V(ngin[0], ngin[1], ngin[2]);
  float cosi = -vdot(d, n);
  float ei = 1.0f, et = ior;
  if (cosi < 0.0f) {
    n = vneg(n);
    cosi = -cosi;
    ei = ior;
    et = 1.0f;
  }
  float F = orc_fresnel(cosi, ei, et);
  v3 nd, side;
  if (u < F) {
    float dn = vdot(d, n);
    nd = V(d.x - n.x * (2.0f * dn), d.y - n.y * (2.0f * dn), d.z - n.z * (2.0f * dn));
    side = n;
  } else {
    float rel = ei / et;
    float sin2t = (rel * rel) * (1.0f - cosi * cosi);
    float cost = sqrtf(1.0f - sin2t);
    float kk = rel * cosi - cost;
    nd = V(d.x * rel + n.x * kk, d.y * rel + n.y * kk, d.z * rel + n.z * kk);
    side = vneg(n);
  }
  nd = vnorm(nd);
  out[0] = nd.x; out[1] = nd.y; out[2] = nd.z;
  side_out[0] = side.x; side_out[1] = side.y; side_out[2] = side.z;
}

static void philox_path(const uint32_t key[2], int pix, int smp, int pair, int tag, int slot,
                        int sub, uint32_t w[4]) {
  uint32_t ctr[4] = {(uint32_t)pix, (uint32_t)smp, (uint32_t)pair,
                     ((uint32_t)tag << 24) | ((uint32_t)slot << 8) | (uint32_t)sub};
  orc_philox4x32_10(ctr, key, w);
}

/* One camera path: pinhole ray, closest hits, next-event estimation at diffuse
 * vertices (point lights, emissive quads), cosine-weighted diffuse bounces,
 * Fresnel-chosen reflection/refraction at dielectric spheres, emission seen
 * from the camera or through specular chains, fixed bounce cap, no roulette. */
static void trace_path(const orc_scene* s, const kstate* k, const uint32_t key[2], int pix,
                       int smp, int pair, int tag, float L[3]) {
  L[0] = L[1] = L[2] = 0.0f;
  int x = pix % s->W, y = pix / s->W;
  uint32_t w[4];
  float jx = 0.5f, jy = 0.5f;
  if (!s->pixel_center) {
    philox_path(key, pix, smp, pair, tag, 0, 0, w);
    jx = orc_u01(w[0]);
    jy = orc_u01(w[1]);
  }
  float px = (float)x + jx, py = (float)y + jy;
  float sx = 2.0f * (px / (float)s->W) - 1.0f;
  float sy = 1.0f - 2.0f * (py / (float)s->H);
  v3 o = vld(s->eye);
  v3 d = vnorm(V(s->fwd[0] + s->right[0] * sx + s->up[0] * sy,
                 s->fwd[1] + s->right[1] * sx + s->up[1] * sy,
                 s->fwd[2] + s->right[2] * sx + s->up[2] * sy));
  float beta[3] = {1.0f, 1.0f, 1.0f};
  int specular = 1;
  for (int v = 0; v <= s->B; ++v) {
    hitrec h;
    closest(s, k, o, d, INFINITY, 0, &h);
    if (h.id < 0) {
      for (int c = 0; c < 3; ++c) L[c] = L[c] + beta[c] * s->env[c];
      break;
    }
    v3 p = vray(o, d, h.t);
    int mat;
    v3 ng;
    prim_info(s, k, h.id, p, &mat, &ng);
    int mt = s->mat_type[mat];
    const float* rgb = k->rgb + 3 * mat;
    if (mt == ORC_EMISSIVE) {
      if (specular && vdot(d, ng) < 0.0f)
        for (int c = 0; c < 3; ++c) L[c] = L[c] + beta[c] * rgb[c];
      break;
    }
    philox_path(key, pix, smp, pair, tag, v + 1, 0, w);
    if (mt == ORC_DIFFUSE) {
      v3 n = vdot(ng, d) > 0.0f ? vneg(ng) : ng;
      float f[3] = {rgb[0] * INV_PI_F, rgb[1] * INV_PI_F, rgb[2] * INV_PI_F};
      for (int l = 0; l < s->n_pl; ++l) {
        const float* lp = k->pl + 6 * l;
        v3 toL = vsub(vld(lp), p);
        float dist2 = vdot(toL, toL);
        float dist = sqrtf(dist2);
        v3 wi = vscale(toL, 1.0f / dist);
        float cx = vdot(n, wi);
        if (!(cx > 0.0f)) continue;
        hitrec hs;
        closest(s, k, spawn(p, n), wi, dist * 0.9999f, 1, &hs);
        if (hs.id >= 0) continue;
        for (int c = 0; c < 3; ++c) L[c] = L[c] + beta[c] * f[c] * ((lp[3 + c] * cx) / dist2);
      }
      int area_rank = 0;
      for (int qi = 0; qi < s->n_quad; ++qi) {
        int qm = s->quad_mat[qi];
        if (s->mat_type[qm] != ORC_EMISSIVE) continue;
        float a, b;
        if (area_rank == 0) {
          a = orc_u01(w[0]);
          b = orc_u01(w[1]);
        } else {
          uint32_t w2[4];
          philox_path(key, pix, smp, pair, tag, v + 1, area_rank, w2);
          a = orc_u01(w2[0]);
          b = orc_u01(w2[1]);
        }
        ++area_rank;
        const float* qd = k->quad + 9 * qi;
        v3 qo = vld(qd), e1 = vld(qd + 3), e2 = vld(qd + 6);
        v3 yl = V(qo.x + e1.x * a + e2.x * b, qo.y + e1.y * a + e2.y * b,
                  qo.z + e1.z * a + e2.z * b);
        v3 nl = vcross(e1, e2);
        float area = sqrtf(vdot(nl, nl));
        v3 nlu = vscale(nl, 1.0f / area);
        v3 toL = vsub(yl, p);
        float dist2 = vdot(toL, toL);
        float dist = sqrtf(dist2);
        v3 wi = vscale(toL, 1.0f / dist);
        float cx = vdot(n, wi);
        float cl = -vdot(nlu, wi);
        if (!(cx > 0.0f && cl > 0.0f)) continue;
        hitrec hs;
        closest(s, k, spawn(p, n), wi, dist * 0.9999f, 1, &hs);
        if (hs.id >= 0) continue;
        float G = ((cx * cl) * area) / dist2;
        const float* le = k->rgb + 3 * qm;
        for (int c = 0; c < 3; ++c) L[c] = L[c] + beta[c] * f[c] * le[c] * G;
      }
      if (v == s->B) break;
      float nin[3] = {n.x, n.y, n.z}, nd[3];
      orc_cosine_direction(nin, orc_u01(w[2]), orc_u01(w[3]), nd);
      o = spawn(p, n);
      d = V(nd[0], nd[1], nd[2]);
      for (int c = 0; c < 3; ++c) beta[c] = beta[c] * rgb[c];
      specular = 0;
    } else { /* dielectric sphere */
      if (v == s->B) break;
      float din[3] = {d.x, d.y, d.z}, nin[3] = {ng.x, ng.y, ng.z}, nd[3], side[3];
      orc_dielectric_scatter(din, nin, s->mat_ior[mat], orc_u01(w[2]), nd, side);
      o = spawn(p, V(side[0], side[1], side[2]));
      d = V(nd[0], nd[1], nd[2]);
      specular = 1;
    }
  }
}

static void render_pixel(const orc_scene* s, const kstate* k, const uint32_t key[2], int pix,
                         int pair, int tag, float out[3]) {
  double acc[3] = {0.0, 0.0, 0.0};
  for (int smp = 0; smp < s->spp; ++smp) {
    float L[3];
    trace_path(s, k, key, pix, smp, pair, tag, L);
    for (int c = 0; c < 3; ++c) acc[c] += (double)L[c];
  }
  for (int c = 0; c < 3; ++c) out[c] = (float)(acc[c] / (double)s->spp);
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

void orc_render(const orc_scene* s, const float* X, int tag, int pair, uint64_t seed,
                int nthreads, float* img) {
  kstate k;
  kstate_init(s, X, &k);
  uint32_t key[2];
  seed_key(seed, key);
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = 0; y < s->H; ++y)
    for (int x = 0; x < s->W; ++x) {
      int pix = y * s->W + x;
      render_pixel(s, &k, key, pix, pair, tag, img + 3 * (size_t)pix);
    }
  kstate_free(&k);
}

void orc_render_pixels(const orc_scene* s, const float* X, int tag, int pair, uint64_t seed,
                       int n, const int32_t* pix, int nthreads, float* out) {
  kstate k;
  kstate_init(s, X, &k);
  uint32_t key[2];
  seed_key(seed, key);
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
  for (int i = 0; i < n; ++i) render_pixel(s, &k, key, pix[i], pair, tag, out + 3 * (size_t)i);
  kstate_free(&k);
}

/* per-image loss: mean over pixels and channels of (I - R)^2 (Eq. 2, MSE) */
double orc_mse(const float* img, const float* ref, int npix) {
  double acc = 0.0;
  for (long i = 0; i < 3L * npix; ++i) {
    double e = (double)img[i] - (double)ref[i];
    acc += e * e;
  }
  return acc / (3.0 * (double)npix);
}

static int check_args(const orc_scene* s, const float* sigma, int N) {
  if (N < 2 || (N & 1)) return -1;
  if (s->n_param < 1 || s->n_param > ORC_MAX_PARAMS) return -1;
  for (int j = 0; j < s->n_param; ++j)
    if (!(sigma[j] > 0.0f) || !isfinite(sigma[j])) return -1;
  return 0;
}

/* renders theta + tau_p (m = 0) and theta - tau_p (m = 1) with the pair's
 * shared path stream and returns per-image losses L[2p+m] */
static void perturbed_losses(const orc_scene* s, const float* ref, const float* theta,
                             const float* tau, int P, uint64_t seed, int nthreads,
                             double* L, float* images) {
  int d = s->n_param;
  size_t npix = (size_t)s->W * (size_t)s->H;
  float* img = images ? NULL : (float*)malloc(sizeof(float) * 3 * npix);
  float X[ORC_MAX_PARAMS];
  for (int p = 0; p < P; ++p)
    for (int m = 0; m < 2; ++m) {
      for (int j = 0; j < d; ++j)
        X[j] = m == 0 ? theta[j] + tau[p * d + j] : theta[j] - tau[p * d + j];
      float* out = images ? images + (size_t)(2 * p + m) * 3 * npix : img;
      orc_render(s, X, ORC_TAG_PATH, p, seed, nthreads, out);
      if (L) L[2 * p + m] = orc_mse(out, ref, (int)npix);
    }
  free(img);
}

/* independent draws: renders theta + tau_i, each with its own path stream i */
static void independent_losses(const orc_scene* s, const float* ref, const float* theta,
                               const float* tau, int N, uint64_t seed, int nthreads,
                               double* L, float* images) {
  int d = s->n_param;
  size_t npix = (size_t)s->W * (size_t)s->H;
  float* img = images ? NULL : (float*)malloc(sizeof(float) * 3 * npix);
  float X[ORC_MAX_PARAMS];
  for (int i = 0; i < N; ++i) {
    for (int j = 0; j < d; ++j) X[j] = theta[j] + tau[i * d + j];
    float* out = images ? images + (size_t)i * 3 * npix : img;
    orc_render(s, X, ORC_TAG_PATH, i, seed, nthreads, out);
    if (L) L[i] = orc_mse(out, ref, (int)npix);
  }
  free(img);
}

int orc_grad_estimate(const orc_scene* s, const float* ref, const float* theta,
                      const float* sigma, int N, uint64_t seed, int mode, int nthreads,
                      double* grad, double* loss, double* losses, float* tau_out) {
  if (check_args(s, sigma, N)) return -1;
  const int indep = (mode & ORC_EST_INDEPENDENT) != 0;
  int P = indep ? N : N / 2, d = s->n_param;
  float* tau = (float*)malloc(sizeof(float) * (size_t)(P * d));
  double* c = (double*)malloc(sizeof(double) * (size_t)(P * d));
  double* L = (double*)malloc(sizeof(double) * (size_t)N);
  if (orc_draw_tau(mode, d, P, seed, sigma, tau, c)) {
    free(tau); free(c); free(L);
    return -1;
  }
  double q;
  if (indep) {
    independent_losses(s, ref, theta, tau, N, seed, nthreads, L, NULL);
    orc_combine_independent(N, d, c, L, grad, &q);
  } else {
    perturbed_losses(s, ref, theta, tau, P, seed, nthreads, L, NULL);
    orc_combine(P, d, c, L, grad, &q);
  }
  if (loss) *loss = q;
  if (losses) memcpy(losses, L, sizeof(double) * (size_t)N);
  if (tau_out) memcpy(tau_out, tau, sizeof(float) * (size_t)(P * d));
  free(tau); free(c); free(L);
  return 0;
}

/* Q estimate with tau drawn from the kernel itself and no extra kernel weight */
int orc_smoothed_loss(const orc_scene* s, const float* ref, const float* theta,
                      const float* sigma, int N, uint64_t seed, int nthreads, double* loss) {
  double* g = (double*)malloc(sizeof(double) * (size_t)(s->n_param > 0 ? s->n_param : 1));
  int rc = orc_grad_estimate(s, ref, theta, sigma, N, seed, ORC_EST_GAUSS, nthreads, g, loss,
                             NULL, NULL);
  free(g);
  return rc;
}

int orc_render_perturbed(const orc_scene* s, const float* theta, const float* sigma, int N,
                         uint64_t seed, int mode, int nthreads, float* images, float* tau_out) {
  if (check_args(s, sigma, N)) return -1;
  const int indep = (mode & ORC_EST_INDEPENDENT) != 0;
  int P = indep ? N : N / 2, d = s->n_param;
  float* tau = (float*)malloc(sizeof(float) * (size_t)(P * d));
  double* c = (double*)malloc(sizeof(double) * (size_t)(P * d));
  if (orc_draw_tau(mode, d, P, seed, sigma, tau, c)) {
    free(tau); free(c);
    return -1;
  }
  if (indep)
    independent_losses(s, NULL, theta, tau, N, seed, nthreads, NULL, images);
  else
    perturbed_losses(s, NULL, theta, tau, P, seed, nthreads, NULL, images);
  if (tau_out) memcpy(tau_out, tau, sizeof(float) * (size_t)(P * d));
  free(tau); free(c);
  return 0;
}

/* linear bandwidth decay (Sec. 3.3) with t normalised to [0, 1] over T steps */
double orc_sigma_schedule(double sigma0, double sigma_end, int t, int T) {
  if (T <= 1) return sigma0;
  return sigma0 + (sigma_end - sigma0) * (double)t / (double)(T - 1);
}

/* Adam (Kingma & Ba, 2015), step t >= 1 */
void orc_adam_step(int d, double* theta, const double* g, double* m, double* v, int t,
                   double lr, double b1, double b2, double eps) {
  for (int j = 0; j < d; ++j) {
    m[j] = b1 * m[j] + (1.0 - b1) * g[j];
    v[j] = b2 * v[j] + (1.0 - b2) * g[j] * g[j];
    double mh = m[j] / (1.0 - pow(b1, t));
    double vh = v[j] / (1.0 - pow(b2, t));
    theta[j] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* ========================================================================= */
/* Eq. 9: the smoothed gradient through a differentiable renderer            */
/* ========================================================================= */
/* For scenes of one diffuse sphere (the parameters move its centre) over one
 * diffuse quad (the ground) lit by one point light, rendered with direct
 * light only.  The pixel value is the box-filtered integral of the point
 * radiance f(x; theta) over the pixel (Sec. 2.1, Eq. 1-3); its derivative
 * (Reynolds transport in the image plane) is
 *     dI/dtheta = int_pixel df/dtheta dx  +  sum over moving edges of
 *                 int_edge (f_inside - f_outside) (v . n_out) dl,
 * the interior term from the shading of the sphere (the hit point and normal
 * move with the centre; the ground's shading does not depend on theta), and
 * edge terms on the two discontinuities that move: the sphere's silhouette
 * and the boundary of its shadow on the ground.  Both edges are closed curves
 * traced by a circle of tangent points on the sphere (seen from the eye, and
 * from the light); they are sampled uniformly in the circle's angle (edge
 * sampling), each sample adding to the pixel it falls in.  The estimator of
 * Eq. 9 with perturbations drawn from the kernel (the kernel weight then
 * drops, as for Eq. 7) is
 *     g = (1/N) sum_k dL/dtheta (theta + tau_k),
 *     dL/dtheta = 2/(3HW) sum_px,c (I_k - R) dI_k/dtheta,
 * with I_k the rendered image and dI_k/dtheta from samples independent of
 * it (interior jitter from stream tag 6, edge angles from tag 7), so that the
 * product estimates the gradient of the loss of the expected image.
 * Per-sample arithmetic is binary32 in a fixed order; sums are binary64. */

#define ORC_TAG_DIFF 6
#define ORC_TAG_EDGE 7
#define DP_SILHOUETTE 1
#define DP_SHADOW 2

/* the scene checks of the differentiable renderer; 0 if supported */
static int dp_supported(const orc_scene* s) {
  if (s->n_sph != 1 || s->n_quad != 1 || s->n_mesh != 0 || s->n_tri != 0 || s->n_pl != 1) return -1;
  if (s->B != 0) return -1;
  if (s->mat_type[s->sph_mat[0]] != ORC_DIFFUSE || s->mat_type[s->quad_mat[0]] != ORC_DIFFUSE) return -1;
  if (s->n_param < 1 || s->n_param > 3) return -1;
  for (int j = 0; j < s->n_param; ++j)
    if (s->binding[3 * j] != ORC_BIND_SPHERE || s->binding[3 * j + 1] != 0) return -1;
  return 0;
}

/* image position (pixel units, x right, y down) of world point X, and the
 * rows of its Jacobian d(px, py)/dX */
static void dp_project(const orc_scene* s, v3 X, float* px, float* py, v3* jx, v3* jy) {
  v3 e = vld(s->eye), f = vld(s->fwd), r = vld(s->right), u = vld(s->up);
  v3 D = vsub(X, e);
  float lam = vdot(D, f), a = vdot(D, r), b = vdot(D, u);
  float rr = vdot(r, r), uu = vdot(u, u);
  float sx = a / (lam * rr), sy = b / (lam * uu);
  float hw = 0.5f * (float)s->W, hh = 0.5f * (float)s->H;
  *px = (sx + 1.0f) * hw;
  *py = (1.0f - sy) * hh;
  /* d sx / dX = (r lam - f a) / (lam^2 rr), d sy / dX = (u lam - f b) / (lam^2 uu) */
  float l2r = (lam * lam) * rr, l2u = (lam * lam) * uu;
  v3 gx = V((r.x * lam - f.x * a) / l2r, (r.y * lam - f.y * a) / l2r, (r.z * lam - f.z * a) / l2r);
  v3 gy = V((u.x * lam - f.x * b) / l2u, (u.y * lam - f.y * b) / l2u, (u.z * lam - f.z * b) / l2u);
  *jx = vscale(gx, hw);
  *jy = vscale(gy, -hh);
}

/* direct radiance (rgb) leaving a diffuse point p with unit normal n toward
 * the viewer, lit by the point light, without a shadow test */
static void dp_shade(const orc_scene* s, const kstate* k, int mat, v3 p, v3 n, float out[3]) {
  const float* lp = k->pl;
  v3 toL = vsub(vld(lp), p);
  float dist2 = vdot(toL, toL);
  float dist = sqrtf(dist2);
  v3 wi = vscale(toL, 1.0f / dist);
  float cx = vdot(n, wi);
  for (int c = 0; c < 3; ++c)
    out[c] = cx > 0.0f ? (k->rgb[3 * mat + c] * INV_PI_F) * ((lp[3 + c] * cx) / dist2) : 0.0f;
}

/* the ground's unit normal, oriented toward the light */
static v3 dp_ground_normal(const kstate* k) {
  v3 n = vnorm(vcross(vld(k->quad + 3), vld(k->quad + 6)));
  if (vdot(n, vsub(vld(k->pl), vld(k->quad))) < 0.0f) n = vneg(n);
  return n;
}

/* radiance seen along a ray that leaves the sphere's silhouette tangentially:
 * the ground behind it (shadowed by the sphere or not), or the environment */
static void dp_behind(const orc_scene* s, const kstate* k, v3 o, v3 d, float out[3]) {
  float t;
  if (!quad_test(o, d, k->quad, INFINITY, &t)) {
    for (int c = 0; c < 3; ++c) out[c] = s->env[c];
    return;
  }
  v3 g = vray(o, d, t);
  v3 n = dp_ground_normal(k);
  v3 toL = vsub(vld(k->pl), g);
  float dist = sqrtf(vdot(toL, toL));
  v3 wi = vscale(toL, 1.0f / dist);
  float ts;
  if (sphere_test(spawn(g, n), wi, k->sph, dist * 0.9999f, &ts)) {
    out[0] = out[1] = out[2] = 0.0f;
    return;
  }
  dp_shade(s, k, s->quad_mat[0], g, n, out);
}

/* One silhouette sample at angle fraction `frac` of a turn: its pixel, the
 * radiance step inside minus outside, the normal speed of the edge in pixels
 * per unit move of each centre axis, and the edge length per radian (pixels).
 * Returns 0 if the sample falls outside the image. */
static int dp_silhouette(const orc_scene* s, const kstate* k, float frac, int* pix, float df[3],
                         float vn[3], float* dl) {
  v3 e = vld(s->eye), c = vld(k->sph);
  float rho = k->sph[3];
  v3 a = vsub(e, c);
  float kk = (rho * rho) / vdot(a, a);
  v3 cs = V(c.x + a.x * kk, c.y + a.y * kk, c.z + a.z * kk);
  float rs = rho * sqrtf(1.0f - kk);
  v3 b1, b2;
  onb(vnorm(a), &b1, &b2);
  float sn, cn;
  orc_sincos_2pi(frac, &sn, &cn);
  v3 p = V(cs.x + (b1.x * cn + b2.x * sn) * rs, cs.y + (b1.y * cn + b2.y * sn) * rs,
           cs.z + (b1.z * cn + b2.z * sn) * rs);
  v3 dp = V((b2.x * cn - b1.x * sn) * rs, (b2.y * cn - b1.y * sn) * rs, (b2.z * cn - b1.z * sn) * rs);
  float px, py;
  v3 jx, jy;
  dp_project(s, p, &px, &py, &jx, &jy);
  if (!(px >= 0.0f && px < (float)s->W && py >= 0.0f && py < (float)s->H)) return 0;
  *pix = (int)py * s->W + (int)px;
  float dx = vdot(jx, dp), dy = vdot(jy, dp);
  *dl = sqrtf(dx * dx + dy * dy);
  v3 n = vscale(vsub(p, c), 1.0f / rho);
  float fin[3], fout[3];
  dp_shade(s, k, s->sph_mat[0], p, n, fin);
  v3 dir = vnorm(vsub(p, e));
  dp_behind(s, k, e, dir, fout);
  for (int ch = 0; ch < 3; ++ch) df[ch] = fin[ch] - fout[ch];
  /* tangency h = |c - e|^2 - ((c - e) . w)^2 - rho^2 of the camera ray w:
   * dh/dc = 2 m with m = c - p = -rho n; along the image, dh/dx =
   * -2 q (m . dd/dx) / |d| with q = (c - e) . w and d the unnormalised ray
   * (the camera's fwd + sx right + sy up) of the image point */
  v3 f = vld(s->fwd), r = vld(s->right), u = vld(s->up);
  v3 pe = vsub(p, e);
  float lam = vdot(pe, f);
  float dlen = sqrtf(vdot(pe, pe)) / lam;
  float q = vdot(vsub(c, e), dir);
  v3 m = vscale(n, -rho);
  float gxx = ((-2.0f * q) / dlen) * (vdot(m, r) * (2.0f / (float)s->W));
  float gyy = ((-2.0f * q) / dlen) * (vdot(m, u) * (-2.0f / (float)s->H));
  float gn = sqrtf(gxx * gxx + gyy * gyy);
  /* outward normal speed of the edge: -(dh/dc) / |dh/dx| = 2 rho n / |dh/dx| */
  vn[0] = (2.0f * rho * n.x) / gn;
  vn[1] = (2.0f * rho * n.y) / gn;
  vn[2] = (2.0f * rho * n.z) / gn;
  return 1;
}

/* One sample of the shadow boundary: the ray from the light tangent to the
 * sphere at angle fraction `frac`, continued to the ground point g; its pixel
 * (if g is on the ground, in front of the camera, inside the image and not
 * hidden by the sphere), the lit radiance at g (the step across the edge),
 * the normal speed of the edge toward the shadow, and the length per radian. */
static int dp_shadow(const orc_scene* s, const kstate* k, float frac, int* pix, float df[3],
                     float vn[3], float* dl) {
  v3 e = vld(s->eye), c = vld(k->sph), L = vld(k->pl);
  float rho = k->sph[3];
  v3 a = vsub(L, c);
  float kk = (rho * rho) / vdot(a, a);
  v3 cs = V(c.x + a.x * kk, c.y + a.y * kk, c.z + a.z * kk);
  float rs = rho * sqrtf(1.0f - kk);
  v3 b1, b2;
  onb(vnorm(a), &b1, &b2);
  float sn, cn;
  orc_sincos_2pi(frac, &sn, &cn);
  v3 t = V(cs.x + (b1.x * cn + b2.x * sn) * rs, cs.y + (b1.y * cn + b2.y * sn) * rs,
           cs.z + (b1.z * cn + b2.z * sn) * rs);
  v3 dt = V((b2.x * cn - b1.x * sn) * rs, (b2.y * cn - b1.y * sn) * rs, (b2.z * cn - b1.z * sn) * rs);
  v3 np = dp_ground_normal(k);
  v3 q0 = vld(k->quad);
  v3 tl = vsub(t, L);
  float den = vdot(tl, np);
  if (!(den < 0.0f)) return 0;
  float lam = vdot(vsub(q0, L), np) / den;
  if (!(lam > 1.0f)) return 0;
  v3 g = vray(L, tl, lam);
  /* on the ground quad */
  v3 e1 = vld(k->quad + 3), e2 = vld(k->quad + 6), nq = vcross(e1, e2);
  float nn = vdot(nq, nq);
  v3 gd = vsub(g, q0);
  float al = vdot(vcross(gd, e2), nq) / nn, be = vdot(vcross(e1, gd), nq) / nn;
  if (al < 0.0f || al > 1.0f || be < 0.0f || be > 1.0f) return 0;
  /* seen by the camera: in front of it, inside the image, not behind the sphere */
  v3 f = vld(s->fwd), r = vld(s->right), u = vld(s->up);
  v3 ge = vsub(g, e);
  float lc = vdot(ge, f);
  if (!(lc > 0.0f)) return 0;
  float px, py;
  v3 jx, jy;
  dp_project(s, g, &px, &py, &jx, &jy);
  if (!(px >= 0.0f && px < (float)s->W && py >= 0.0f && py < (float)s->H)) return 0;
  float gdist = sqrtf(vdot(ge, ge));
  v3 wc = vscale(ge, 1.0f / gdist);
  float tsp;
  if (sphere_test(e, wc, k->sph, gdist * 0.9999f, &tsp)) return 0;
  *pix = (int)py * s->W + (int)px;
  /* d g / d angle: the ray parameter lam changes with t */
  float dlam = -lam * (vdot(dt, np) / den);
  v3 dg = V(dt.x * lam + tl.x * dlam, dt.y * lam + tl.y * dlam, dt.z * lam + tl.z * dlam);
  float dx = vdot(jx, dg), dy = vdot(jy, dg);
  *dl = sqrtf(dx * dx + dy * dy);
  dp_shade(s, k, s->quad_mat[0], g, np, df);
  /* tangency of the light ray: h = |c - L|^2 - ((c - L) . w)^2 - rho^2 with w
   * the unit direction from L to g; dh/dc = 2 m_s, m_s = (c - L) - q_s w;
   * along the image, dh/dx = -2 q_s (m_s . dg/dx) / |g - L| with
   * dg/dx = lc [dd/dx - ((dd/dx . np) / (d . np)) d], d = (g - e) / lc */
  v3 lg = vsub(g, L);
  float lgd = sqrtf(vdot(lg, lg));
  v3 w = vscale(lg, 1.0f / lgd);
  v3 cl = vsub(c, L);
  float qs = vdot(cl, w);
  v3 ms = V(cl.x - w.x * qs, cl.y - w.y * qs, cl.z - w.z * qs);
  v3 d = vscale(ge, 1.0f / lc);
  float dn = vdot(d, np);
  v3 ddx = vscale(r, 2.0f / (float)s->W), ddy = vscale(u, -2.0f / (float)s->H);
  float ax = vdot(ddx, np) / dn, ay = vdot(ddy, np) / dn;
  v3 dgx = V((ddx.x - d.x * ax) * lc, (ddx.y - d.y * ax) * lc, (ddx.z - d.z * ax) * lc);
  v3 dgy = V((ddy.x - d.x * ay) * lc, (ddy.y - d.y * ay) * lc, (ddy.z - d.z * ay) * lc);
  float gxx = ((-2.0f * qs) * vdot(ms, dgx)) / lgd;
  float gyy = ((-2.0f * qs) * vdot(ms, dgy)) / lgd;
  float gn = sqrtf(gxx * gxx + gyy * gyy);
  /* the lit side's outward normal points into the shadow, where h < 0:
   * speed (dh/dc) / |dh/dx| = 2 m_s / |dh/dx| */
  vn[0] = (2.0f * ms.x) / gn;
  vn[1] = (2.0f * ms.y) / gn;
  vn[2] = (2.0f * ms.z) / gn;
  return 1;
}

/* Interior derivative sample at image point (px, py): df/dc (rgb x centre
 * axis) if the camera ray meets the sphere first, else 0 (the ground's
 * shading does not depend on the sphere away from the shadow's edge). */
static void dp_interior(const orc_scene* s, const kstate* k, float px, float py, float out[3][3]) {
  for (int c = 0; c < 3; ++c)
    for (int j = 0; j < 3; ++j) out[c][j] = 0.0f;
  float sx = 2.0f * (px / (float)s->W) - 1.0f;
  float sy = 1.0f - 2.0f * (py / (float)s->H);
  v3 e = vld(s->eye);
  v3 d = vnorm(V(s->fwd[0] + s->right[0] * sx + s->up[0] * sy,
                 s->fwd[1] + s->right[1] * sx + s->up[1] * sy,
                 s->fwd[2] + s->right[2] * sx + s->up[2] * sy));
  float ts, tg;
  if (!sphere_test(e, d, k->sph, INFINITY, &ts)) return;
  if (quad_test(e, d, k->quad, ts, &tg)) return;  /* the ground is nearer */
  v3 c = vld(k->sph);
  float rho = k->sph[3];
  v3 p = vray(e, d, ts);
  v3 n = vscale(vsub(p, c), 1.0f / rho);
  v3 v = vsub(vld(k->pl), p);
  float nv = vdot(n, v);
  if (!(nv > 0.0f)) return;
  float r2 = vdot(v, v), rr = sqrtf(r2), r3 = r2 * rr;
  float dn = vdot(d, n);
  const int mat = s->sph_mat[0];
  for (int j = 0; j < 3; ++j) {
    /* the hit moves along the ray: dt/dc_j = n_j / (d . n) */
    float nj = j == 0 ? n.x : j == 1 ? n.y : n.z;
    float dtj = nj / dn;
    v3 dpj = vscale(d, dtj);
    v3 ej = V(j == 0 ? 1.0f : 0.0f, j == 1 ? 1.0f : 0.0f, j == 2 ? 1.0f : 0.0f);
    v3 dnj = vscale(vsub(dpj, ej), 1.0f / rho);
    /* d/dc_j of (n . v) / |v|^3 with dv = -dp */
    float dnv = vdot(dnj, v) - vdot(n, dpj);
    float dvv = -vdot(v, dpj);
    float dg = dnv / r3 - ((3.0f * nv) * dvv) / (r2 * r3);
    for (int ch = 0; ch < 3; ++ch)
      out[ch][j] = (k->rgb[3 * mat + ch] * INV_PI_F) * (k->pl[3 + ch] * dg);
  }
}

/* dI/dtheta of one render (params X, stream pair `pair`): out[H][W][3][d]
 * (binary64), the terms selected by mask (1 interior, 2 silhouette, 4 shadow);
 * spp interior samples per pixel, edge_samples samples per edge. */
int orc_dp_image_derivative(const orc_scene* s, const float* X, int pair, uint64_t seed,
                            int edge_samples, int mask, int nthreads, double* out) {
  if (dp_supported(s) || edge_samples < 1) return -1;
  const int d = s->n_param, W = s->W, H = s->H;
  kstate k;
  kstate_init(s, X, &k);
  uint32_t key[2];
  seed_key(seed, key);
  set_threads(nthreads);
  memset(out, 0, sizeof(double) * (size_t)W * H * 3 * d);
  if (mask & 1) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int pix = 0; pix < W * H; ++pix) {
      double acc[3][3] = {{0}};
      for (int smp = 0; smp < s->spp; ++smp) {
        float jx = 0.5f, jy = 0.5f;
        if (!s->pixel_center) {
          uint32_t w[4];
          philox_path(key, pix, smp, pair, ORC_TAG_DIFF, 0, 0, w);
          jx = orc_u01(w[0]);
          jy = orc_u01(w[1]);
        }
        float px = (float)(pix % W) + jx, py = (float)(pix / W) + jy;
        float g[3][3];
        dp_interior(s, &k, px, py, g);
        for (int c = 0; c < 3; ++c)
          for (int j = 0; j < 3; ++j) acc[c][j] += (double)g[c][j];
      }
      for (int c = 0; c < 3; ++c)
        for (int j = 0; j < d; ++j) {
          int ax = s->binding[3 * j + 2];
          out[((size_t)pix * 3 + c) * d + j] = acc[c][ax] / (double)s->spp;
        }
    }
  }
  for (int edge = 0; edge < 2; ++edge) {
    if (!(mask & (edge == 0 ? 2 : 4))) continue;
    for (int m = 0; m < edge_samples; ++m) {
      uint32_t ctr[4] = {(uint32_t)m, (uint32_t)edge, (uint32_t)pair,
                         (uint32_t)ORC_TAG_EDGE << 24};
      uint32_t w[4];
      orc_philox4x32_10(ctr, key, w);
      float frac = ((float)m + orc_u01(w[0])) / (float)edge_samples;
      int pix;
      float df[3], vn[3], dl;
      int ok = edge == 0 ? dp_silhouette(s, &k, frac, &pix, df, vn, &dl)
                         : dp_shadow(s, &k, frac, &pix, df, vn, &dl);
      if (!ok) continue;
      /* the sample stands for 2 pi / M radians of the edge */
      double wgt = (2.0 * ORC_PI / (double)edge_samples) * (double)dl;
      for (int c = 0; c < 3; ++c)
        for (int j = 0; j < d; ++j) {
          int ax = s->binding[3 * j + 2];
          out[((size_t)pix * 3 + c) * d + j] += wgt * (double)df[c] * (double)vn[ax];
        }
    }
  }
  kstate_free(&k);
  return 0;
}

/* Eq. 9 estimate: tau_k from the kernel (antithetic GAUSS pairs), renders
 * I_k at theta +- tau_p (path stream of pair p), dI_k/dtheta with the
 * derivative streams of pair p, and
 *     g = (1/N) sum_k 2/(3HW) sum (I_k - R) dI_k/dtheta,  Q = mean L_k. */
int orc_dp_grad_estimate(const orc_scene* s, const float* ref, const float* theta,
                         const float* sigma, int N, uint64_t seed, int edge_samples, int nthreads,
                         double* grad, double* loss, double* losses) {
  if (check_args(s, sigma, N) || dp_supported(s) || edge_samples < 1) return -1;
  const int d = s->n_param, P = N / 2;
  const size_t npix = (size_t)s->W * s->H;
  float* tau = (float*)malloc(sizeof(float) * (size_t)(P * d));
  double* c = (double*)malloc(sizeof(double) * (size_t)(P * d));
  float* img = (float*)malloc(sizeof(float) * 3 * npix);
  double* dimg = (double*)malloc(sizeof(double) * 3 * npix * (size_t)d);
  double* L = (double*)malloc(sizeof(double) * (size_t)N);
  orc_draw_tau(ORC_EST_GAUSS, d, P, seed, sigma, tau, c);
  for (int j = 0; j < d; ++j) grad[j] = 0.0;
  float X[ORC_MAX_PARAMS];
  for (int p = 0; p < P; ++p)
    for (int mm = 0; mm < 2; ++mm) {
      for (int j = 0; j < d; ++j)
        X[j] = mm == 0 ? theta[j] + tau[p * d + j] : theta[j] - tau[p * d + j];
      orc_render(s, X, ORC_TAG_PATH, p, seed, nthreads, img);
      L[2 * p + mm] = orc_mse(img, ref, (int)npix);
      orc_dp_image_derivative(s, X, p, seed, edge_samples, 7, nthreads, dimg);
      const double scale = 2.0 / (3.0 * (double)npix);
      for (int j = 0; j < d; ++j) {
        double acc = 0.0;
        for (size_t i = 0; i < 3 * npix; ++i)
          acc += ((double)img[i] - (double)ref[i]) * dimg[i * d + j];
        grad[j] += scale * acc;
      }
    }
  double q = 0.0;
  for (int i = 0; i < N; ++i) q += L[i];
  for (int j = 0; j < d; ++j) grad[j] /= (double)N;
  if (loss) *loss = q / (double)N;
  if (losses) memcpy(losses, L, sizeof(double) * (size_t)N);
  free(tau); free(c); free(img); free(dimg); free(L);
  return 0;
}
