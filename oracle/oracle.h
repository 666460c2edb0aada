/*
 * CPU oracle for the plateau-reduced gradient estimator (Fischer & Ritschel,
 * "Plateau-reduced Differentiable Path Tracing", CVPR 2023).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load this library.  It shares no code with the HIP path.
 *
 * Numerics: per-sample geometry and radiance are evaluated in IEEE binary32 with
 * a fixed operation order and no contraction, because the hit tests decide which
 * primitive a ray hits (an integer) and that decision is taken in the precision
 * of the GPU path.  Pixel averages, image losses and the gradient combination are
 * accumulated in binary64.
 */
#ifndef PRDPT_ORACLE_H
#define PRDPT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_DIFFUSE = 0, ORC_DIELECTRIC = 1, ORC_EMISSIVE = 2 };
#define ORC_MAX_PARAMS 256

enum { ORC_BIND_SPHERE = 0, ORC_BIND_QUAD = 1, ORC_BIND_MESH = 2, ORC_BIND_PLIGHT = 3,
       ORC_BIND_ALBEDO = 4, /* material colour channel: albedo (diffuse) or radiance (emissive) */
       ORC_BIND_MESH_ROT = 5 /* mesh rotation angle (radians) about the x, y or z axis */ };
enum { ORC_EST_GAUSS = 0, ORC_EST_IS = 1, ORC_EST_IS_PERDIM = 2 };
/* flag or-ed into a mode: independent perturbations without the antithetic
 * partner (the paper's noAT ablation, Sec. 4.4, Tab. 4): N draws, one render each at
 * theta + tau_i with its own path stream, single-sample score weights */
enum { ORC_EST_INDEPENDENT = 0x100 };
/* flag or-ed into an independent mode: stratified draws, the alternative to
 * antithetic pairs that Sec. 3.2 mentions; the first uniform of draw i of P is
 * moved into stratum i, (i + u) / P, so the P draws cover [0, 1) once each */
enum { ORC_EST_STRATIFIED = 0x200 };
enum { ORC_TAG_TAU = 1, ORC_TAG_PATH = 2, ORC_TAG_REF = 3 };

/* Scene as flat arrays; the oracle copies everything it needs. */
typedef struct {
  float eye[3], fwd[3], right[3], up[3];
  int32_t width, height, spp, max_bounces, pixel_center;
  float env[3];
  int32_t n_mat;   const int32_t* mat_type; const float* mat_rgb; const float* mat_ior;
  int32_t n_sph;   const float* sph;  const int32_t* sph_mat;      /* [n][4] cx cy cz r */
  int32_t n_quad;  const float* quad; const int32_t* quad_mat;     /* [n][9] o e1 e2 */
  int32_t n_mesh;  const int32_t* mesh_off; const int32_t* mesh_mat; const float* mesh_xlate;
  int32_t n_tri;   const float* tri;                               /* [n][9] v0 v1 v2 */
  int32_t n_plight; const float* plight;                           /* [n][6] pos rgb */
  int32_t n_param; const int32_t* binding;                         /* [d][3] */
  const float* mesh_rot;   /* [n_mesh][3] angles (a, b, c) or NULL (all zero): a mesh's
                              vertex x maps to R x + translation, R = Rz(c) Ry(b) Rx(a) */
} orc_scene_in;

typedef struct orc_scene orc_scene;

/* counter-based generator and sample transforms */
void  orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
float orc_u01(uint32_t x);
float orc_ln(float x);
void  orc_sincos_2pi(float u, float* s, float* c);
double orc_chi_mean(int d);

/* perturbation draw: tau[P][d] (binary32) and pair weights c[P][d] (binary64) */
int orc_draw_tau(int mode, int d, int P, uint64_t seed, const float* sigma,
                 float* tau, double* c);
/* g_j = (1/P) sum_p c[p][j] (L[2p] - L[2p+1]);  q = mean of L over 2P */
void orc_combine(int P, int d, const double* c, const double* L, double* g, double* q);
/* independent draws: g_j = (1/N) sum_i c_ij L_i, q = mean L */
void orc_combine_independent(int N, int d, const double* c, const double* L, double* g,
                             double* q);

/* scene */
orc_scene* orc_scene_new(const orc_scene_in* in);
void orc_scene_free(orc_scene* s);
void orc_set_brute_force(orc_scene* s, int on);
/* closest hit of n rays (o, d): t (inf on miss) and primitive id (-1) at params X */
void orc_trace(const orc_scene* s, const float* X, int n, const float* o, const float* d,
               float* t_out, int32_t* id_out);
/* render the full image at params X with stream tag/pair/seed -> img[H][W][3] */
void orc_render(const orc_scene* s, const float* X, int tag, int pair, uint64_t seed,
                int nthreads, float* img);
/* render listed pixels (index y*W+x) -> out[n][3] */
void orc_render_pixels(const orc_scene* s, const float* X, int tag, int pair, uint64_t seed,
                       int n, const int32_t* pix, int nthreads, float* out);
double orc_mse(const float* img, const float* ref, int npix);

/* estimator: returns 0, or -1 on invalid arguments */
int orc_grad_estimate(const orc_scene* s, const float* ref, const float* theta,
                      const float* sigma, int N, uint64_t seed, int mode, int nthreads,
                      double* grad, double* loss, double* losses, float* tau);
int orc_smoothed_loss(const orc_scene* s, const float* ref, const float* theta,
                      const float* sigma, int N, uint64_t seed, int nthreads, double* loss);
int orc_render_perturbed(const orc_scene* s, const float* theta, const float* sigma, int N,
                         uint64_t seed, int mode, int nthreads, float* images, float* tau);

/* scattering steps of the path tracer, exposed for closed-form checks:
 * unpolarised Fresnel reflectance; the cosine-weighted diffuse direction about
 * a unit normal from two uniforms; the dielectric interface (reflect with
 * probability F chosen by u, else refract by Snell's law), returning the unit
 * new direction and the normal of the side the next origin is offset to */
float orc_fresnel(float cos_i, float eta_i, float eta_t);
void orc_cosine_direction(const float n[3], float u1, float u2, float out[3]);
void orc_dielectric_scatter(const float d[3], const float ng[3], float ior, float u,
                            float out[3], float side[3]);

/* Eq. 9 through a differentiable direct-light renderer (scenes of one
 * diffuse sphere, bound by its centre, over one diffuse quad under one point
 * light, no bounces): the derivative image dI/dtheta [H][W][3][d] of one
 * render (mask: 1 interior, 2 silhouette edge, 4 shadow edge; spp interior
 * samples per pixel, edge_samples per edge), and the estimate
 * g = (1/N) sum_k 2/(3HW) sum (I_k - R) dI_k/dtheta over antithetic GAUSS
 * perturbations.  Return -1 on unsupported scenes or arguments. */
int orc_dp_image_derivative(const orc_scene* s, const float* X, int pair, uint64_t seed,
                            int edge_samples, int mask, int nthreads, double* out);
int orc_dp_grad_estimate(const orc_scene* s, const float* ref, const float* theta,
                         const float* sigma, int N, uint64_t seed, int edge_samples, int nthreads,
                         double* grad, double* loss, double* losses);

/* optimiser helpers (host-side step of the optimisation loop) */
double orc_sigma_schedule(double sigma0, double sigma_end, int t, int T);
void orc_adam_step(int d, double* theta, const double* g, double* m, double* v, int t,
                   double lr, double b1, double b2, double eps);

#ifdef __cplusplus
}
#endif
#endif
