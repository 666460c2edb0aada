/*
 * prdpt.h — C ABI of the MI355X (gfx950) plateau-reduced gradient estimator.
 *
 * The library evaluates, on one GPU, the Monte Carlo gradient of the
 * kernel-smoothed inverse-rendering objective of Fischer & Ritschel,
 * "Plateau-reduced Differentiable Path Tracing" (CVPR 2023):
 *
 *     Q(theta)   = integral kappa_sigma(tau) L(theta + tau) dtau            (Sec. 3.1, Eq. 6)
 *     grad Q     ~ (1/N) sum_i dkappa/dtheta(tau_i) L(theta - tau_i)          (Sec. 3.1, Eq. 10)
 *     L(theta)   = mean over pixels and RGB of (I_theta - R)^2               (Sec. 2.1, Eq. 2; Sec. 4.1 MSE)
 *
 * with a Gaussian kernel kappa = N(0, diag sigma^2) (supplement, kernel
 * definition), antithetic pairs tau / -tau and importance sampling of the
 * positivised kernel derivative (Sec. 3.2).  The renderer I_theta is this
 * library's own path tracer, treated by the estimator as a black box, as the
 * paper treats its renderer (Sec. 3.1, "if P is not differentiable").
 *
 * Conventions for every call:
 *   - Status codes: PRDPT_OK (0) or a negative PRDPT_E_* value.  Nothing throws
 *     across the ABI.  prdpt_last_error() returns a thread-local message for
 *     the last failing call on the calling thread.
 *   - N is the number of perturbed renders, 2 x (antithetic pairs); it must be
 *     even and >= 2.  Perturbation index k = 2p + m: m = 0 renders theta + tau_p,
 *     m = 1 renders theta - tau_p; both share the pair's path-sample stream.
 *     (With PRDPT_EST_INDEPENDENT: render k is theta + tau_k, stream k.)
 *   - theta and sigma have length d = the scene's parameter count; sigma_j > 0.
 *   - "host" pointers are ordinary CPU memory, "device" pointers are HIP device
 *     memory of the context's device.  Outputs are owned by the caller.
 *   - Results are a pure function of (scene description, ref, theta, sigma, N,
 *     seed, est): they do not depend on the context, the stream, batching or
 *     device load.
 *   - A context binds one device and one HIP stream; calls on one context are
 *     serialised by the library; calls on different contexts may run from
 *     different threads.
 */
#ifndef PRDPT_H
#define PRDPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define PRDPT_OK 0
#define PRDPT_E_ARG (-1)       /* null pointer, odd/small N, sigma <= 0, size 0, bad mode */
#define PRDPT_E_NOMEM (-2)     /* device or host allocation failed */
#define PRDPT_E_ADMISSION (-3) /* the scene does not fit the context's HBM budget */
#define PRDPT_E_HIP (-4)       /* a HIP runtime call failed */
#define PRDPT_E_SCENE (-5)     /* invalid scene description */
#define PRDPT_E_CANCELLED (-6) /* request cancelled before it ran */
#define PRDPT_E_TIMEOUT (-7)   /* request did not finish within its deadline */

/* ---- estimator modes (Sec. 3.2) ------------------------------------------ */
/* GAUSS: tau ~ kappa, pair weight z_j / (2 sigma_j); unbiased for grad Q.      */
/* IS: importance sampling of |grad kappa|: radius chi_{d+1}, uniform direction */
/*     (d = 1: the paper's inverse CDF sqrt(-2 sigma^2 ln xi)); pair weight     */
/*     C_d u_j / (2 sigma_j), C_d = mean of chi_d; unbiased for grad Q.         */
/* IS_PERDIM: independent two-sided Rayleigh per axis (literal per-dimension    */
/*     reading); exact for d = 1, biased for non-separable objectives in d > 1. */
/*     Axis j takes its sign from bit j mod 32 of sign word j / 32.             */
#define PRDPT_EST_GAUSS 0
#define PRDPT_EST_IS 1
#define PRDPT_EST_IS_PERDIM 2
/* Flag or-ed into a mode: independent perturbations without the antithetic
 * partner (the paper's noAT ablation, Sec. 4.4, Tab. 4): the N renders are theta +
 * tau_i for N independent draws, each with its own path-sample stream, and
 *     grad_j = (1/N) sum_i c_ij L(theta + tau_i)
 * with the single-sample weights c_ij (twice the pair weights).  Accepted by
 * the single-request calls; the batched and served forms reject it. */
#define PRDPT_EST_INDEPENDENT 0x100
/* Flag or-ed into an independent mode (PRDPT_EST_INDEPENDENT must be set):
 * stratified draws, the alternative to antithetic pairs that Sec. 3.2
 * mentions.  Only the first uniform of draw i of the N draws is moved into
 * stratum i, (i + u) / N (binary32, kept below 1).  For d = 1 that stratifies
 * the IS radius (the whole draw up to its sign); for IS with d > 1 it is one
 * of the (d + 1) / 2 log-uniform terms of the squared radius and the
 * direction is not stratified; for IS_PERDIM it is axis 0's radius; for GAUSS
 * the first Box-Muller radius.  Weights and renders are those of the
 * independent draws.  Accepted by the single-request calls; the batched and
 * served forms reject it. */
#define PRDPT_EST_STRATIFIED 0x200

/* ---- scene description ---------------------------------------------------- */
#define PRDPT_MAT_DIFFUSE 0    /* rgb = albedo; Lambertian */
#define PRDPT_MAT_DIELECTRIC 1 /* ior; smooth glass, spheres only */
#define PRDPT_MAT_EMISSIVE 2   /* rgb = radiance; quads only (one-sided area lights) */

#define PRDPT_BIND_SPHERE 0 /* sphere centre component */
#define PRDPT_BIND_QUAD 1   /* quad origin component */
#define PRDPT_BIND_MESH 2   /* mesh translation component */
#define PRDPT_BIND_PLIGHT 3 /* point-light position component */
#define PRDPT_BIND_ALBEDO 4 /* material colour channel: albedo of a diffuse material,
                               radiance of an emissive one */
#define PRDPT_BIND_MESH_ROT 5 /* mesh rotation angle (radians) about the x, y or z axis */

/* Limits of one scene. */
#define PRDPT_MAX_PARAMS 256
#define PRDPT_BATCH_MAX_PARAMS PRDPT_MAX_PARAMS /* d limit of the batched and served forms */
#define PRDPT_MAX_MATERIALS 32
#define PRDPT_MAX_SPHERES 128
#define PRDPT_MAX_QUADS 16
#define PRDPT_MAX_INSTANCES 8
#define PRDPT_MAX_POINT_LIGHTS 8
#define PRDPT_MAX_BOUNCES 64
#define PRDPT_MAX_SIDE 4096

/*
 * All arrays are host memory, copied by prdpt_scene_create (the caller may free
 * them on return).  Primitive ids, used to break ties between equal hit
 * distances, are: spheres 0..S-1, quads S..S+Q-1, then triangles in array order.
 * Camera: pinhole at eye; the unnormalised direction of image point (sx, sy) in
 * [-1,1]^2 is fwd + sx*right + sy*up (right/up pre-scaled by the field of view;
 * row 0 is the top, sy = +1).  A parameter binding (kind, index, component)
 * makes that scalar field equal its base value plus theta_j.  A mesh is an
 * instance: its vertex x is placed at R x + t, with t its translation and
 * R = Rz(c) Ry(b) Rx(a) for its rotation angles (a, b, c) (rotations about the
 * fixed x, y, z axes through the mesh's origin, applied in that order, formed
 * in binary64 and rounded to binary32); rays are taken into the mesh's static
 * BVH by R^T (o - t) and R^T d.
 */
typedef struct {
  float eye[3], fwd[3], right[3], up[3];
  int32_t width, height;      /* image size, 1..PRDPT_MAX_SIDE */
  int32_t spp;                /* samples per pixel, >= 1 */
  int32_t max_bounces;        /* scattering events after the primary hit, 0..64 */
  int32_t pixel_center;       /* 1: sample pixel centres instead of jittering */
  float env[3];               /* constant environment radiance on misses (normally 0) */
  int32_t n_materials;
  const int32_t* mat_type;    /* [n_materials] PRDPT_MAT_* */
  const float* mat_rgb;       /* [n_materials][3] */
  const float* mat_ior;       /* [n_materials] */
  int32_t n_spheres;
  const float* spheres;       /* [n][4] centre xyz, radius */
  const int32_t* sphere_mat;  /* [n] */
  int32_t n_quads;
  const float* quads;         /* [n][9] origin, edge1, edge2 (normal = edge1 x edge2) */
  const int32_t* quad_mat;    /* [n] */
  int32_t n_meshes;
  const int32_t* mesh_offset; /* [n_meshes + 1] first triangle of each mesh */
  const int32_t* mesh_mat;    /* [n_meshes] */
  const float* mesh_translation; /* [n_meshes][3] */
  int32_t n_triangles;
  const float* triangles;     /* [n_triangles][9] v0, v1, v2 */
  int32_t n_point_lights;
  const float* point_lights;  /* [n][6] position, intensity rgb */
  int32_t n_params;           /* d, 1..PRDPT_MAX_PARAMS */
  const int32_t* bindings;    /* [d][3] kind, index, component */
  const float* mesh_rotation; /* [n_meshes][3] angles (a, b, c) in radians, or NULL (zero) */
} prdpt_scene_desc;

typedef struct prdpt_ctx prdpt_ctx;
typedef struct prdpt_scene prdpt_scene;

/* Thread-local description of the last error on this thread ("" if none). */
const char* prdpt_last_error(void);

/*
 * Create a context on HIP device `device`.  `stream` is the hipStream_t the
 * context enqueues on (NULL: the device's null stream; the stream stays owned
 * by the caller and must outlive the context).  `hbm_budget` bounds the
 * sum of resident scene footprints in bytes (0 = unbounded): scene creation
 * beyond it fails with PRDPT_E_ADMISSION.  Scratch that the context allocates
 * on first use and keeps until it is destroyed is not counted: per-estimate
 * arrays of O(N d + N tiles) elements (N tiles: 4 bytes per perturbation and
 * pixel tile), allocated with 50 % slack.  A scene renders in tiles of 8x8
 * pixels, or of 4x4 pixels when its image has fewer than 2048 8x8 tiles and
 * at least 16 samples per pixel (more, smaller work items for the persistent
 * render kernel); the choice depends on the scene alone, so every entry point
 * and the batched and served forms render a scene the same way.
 */
int prdpt_ctx_create(int device, void* stream, size_t hbm_budget, prdpt_ctx** out);
/* Synchronise and release the context's own memory (scenes must be destroyed first). */
int prdpt_ctx_destroy(prdpt_ctx* ctx);
/* Rebind the context to another stream of the same device (NULL = null stream). */
int prdpt_ctx_set_stream(prdpt_ctx* ctx, void* stream);
/* Bytes currently held by resident scenes of this context. */
int prdpt_ctx_resident_bytes(prdpt_ctx* ctx, size_t* bytes);

/*
 * The scene handle stands for the function P of Alg. 1 (Sec. 3.4): the scene
 * whose image the renderer computes for parameters theta, the pixel integral of
 * Sec. 2.1 (Eq. 1-3), here with the parameter bindings that map theta onto the
 * scene.  Validate and copy a scene, build its BVHs on the host (binned SAH,
 * 4-wide 128-byte nodes, 48-byte triangles and a 4-byte id-to-position entry
 * per triangle), upload them, and return a handle that stays resident in HBM
 * until prdpt_scene_destroy.  *footprint_bytes (nullable)
 * receives the device bytes held.  Errors: PRDPT_E_ARG (null), PRDPT_E_SCENE
 * (limits, indices, material rules), PRDPT_E_ADMISSION, PRDPT_E_NOMEM.
 */
int prdpt_scene_create(prdpt_ctx* ctx, const prdpt_scene_desc* desc, prdpt_scene** out,
                       size_t* footprint_bytes);
int prdpt_scene_destroy(prdpt_scene* scene);
/* width, height, spp, max_bounces, n_params (any may be NULL). */
int prdpt_scene_info(const prdpt_scene* scene, int* width, int* height, int* spp,
                     int* max_bounces, int* n_params);

/*
 * Perturbation draw only (Sec. 3.2): tau_out (host, float[P][d]) and pair weights
 * c_out (host, double[P][d]) of `est` for P pairs (P independent draws and
 * their single-sample weights with PRDPT_EST_INDEPENDENT).  d <= PRDPT_MAX_PARAMS.
 */
int prdpt_draw_tau(prdpt_ctx* ctx, int est, int d, int P, uint64_t seed, const float* sigma,
                   float* tau_out, double* c_out);

/*
 * Render the N perturbed scenes theta +- tau_p (Eq. 6 / Eq. 10 arguments).
 * images_out: device float[N][H][W][3] (k = 2p + m), caller-owned.
 * tau_out: host float[N/2][d] (float[N][d] with PRDPT_EST_INDEPENDENT) or
 * NULL.  Synchronous.
 */
int prdpt_render_perturbed(prdpt_scene* scene, const float* theta, const float* sigma, int N,
                           uint64_t seed, int est, float* images_out, float* tau_out);

/*
 * Render one image at parameters X (host float[d]) with the reference stream
 * (stream tag 3, pair 0) into image_out (device float[H][W][3]).  Used to build
 * reference images R(theta_ref) for Eq. 2.  Synchronous.
 */
int prdpt_render_reference(prdpt_scene* scene, const float* X, uint64_t seed, float* image_out);

/*
 * Monte Carlo estimate of the smoothed objective Q (Eq. 7 read with tau ~ kappa
 * and no extra kernel weight): the mean of the N per-image losses with GAUSS
 * perturbations.  ref: device float[H][W][3].  loss_out: host double.
 */
int prdpt_smoothed_loss(prdpt_scene* scene, const float* ref, const float* theta,
                        const float* sigma, int N, uint64_t seed, double* loss_out);

/*
 * Plateau-reduced gradient (Eq. 10 with antithetic pairs; Alg. 1 with the
 * kernel constant made explicit):
 *     grad_j = (1/P) sum_p c_pj (L(theta + tau_p) - L(theta - tau_p)),
 * accumulated in binary64.  ref: device float[H][W][3].  grad_out: host
 * double[d].  loss_out (nullable): host double, mean of the N losses.
 * losses_out (nullable): host double[N] per-image losses.  Synchronous.
 */
int prdpt_grad_estimate(prdpt_scene* scene, const float* ref, const float* theta,
                        const float* sigma, int N, uint64_t seed, int est, double* grad_out,
                        double* loss_out, double* losses_out);

/*
 * The smoothed gradient through a differentiable renderer (Sec. 3.1, Eq. 9):
 *     grad = (1/N) sum_k dL/dtheta (theta + tau_k),
 *     dL/dtheta = 2/(3 H W) sum over pixels and RGB of (I_k - R) dI_k/dtheta,
 * with tau_k drawn from the kernel (GAUSS antithetic pairs; the kernel weight
 * then drops, as for Eq. 7), I_k the rendered image of perturbation k and
 * dI_k/dtheta from samples independent of it: per pixel, spp interior samples
 * of the shading derivative (stream tag 6), plus edge_samples samples on each
 * of the two edges that move with the parameters, the sphere's silhouette and
 * its shadow's boundary on the ground (stream tag 7, Reynolds transport of
 * the pixel integral).  Supported scenes (else PRDPT_E_SCENE): one diffuse
 * sphere whose centre components are the parameters (d <= 3), one diffuse
 * quad (the ground; the light and the sphere above its plane, the eye too),
 * one point light, no meshes, max_bounces = 0.  ref: device float[H][W][3];
 * grad_out host double[d]; loss_out (nullable) the mean of the N losses;
 * losses_out (nullable) host double[N].  Synchronous.
 */
int prdpt_grad_estimate_dp(prdpt_scene* scene, const float* ref, const float* theta,
                           const float* sigma, int N, uint64_t seed, int edge_samples,
                           double* grad_out, double* loss_out, double* losses_out);

/*
 * Stream-ordered form of prdpt_grad_estimate for callers that keep everything
 * on the device (the torch binding): theta_dev/sigma_dev device float[d];
 * grad_dev device double[d]; loss_dev device double[1]; losses_dev (nullable)
 * device double[N]; c_dev (nullable) device double[N/2][d] receives the pair
 * weights (double[N][d], the single-sample weights, with
 * PRDPT_EST_INDEPENDENT).  Enqueued on the context's stream; no host
 * synchronisation.
 */
int prdpt_grad_estimate_async(prdpt_scene* scene, const float* ref_dev, const float* theta_dev,
                              const float* sigma_dev, int N, uint64_t seed, int est,
                              double* grad_dev, double* loss_dev, double* losses_dev,
                              double* c_dev);

/*
 * Allocation-free form of prdpt_grad_estimate_async, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, results and stream order;
 * the call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine) and records no timing events.  Its scratch lives in a fixed device
 * array of PRDPT_NOALLOC_SCRATCH_BYTES that the library reserves on every
 * device it runs on (looked up when a context is created there) and keeps
 * until the process ends.  A request needs, each rounded up to 256 bytes:
 * N d floats (parameter rows), R d floats (draws) and, if c_dev is NULL, R d
 * doubles (weights), with R = N/2 (R = N with PRDPT_EST_INDEPENDENT); N x
 * tiles floats (tile losses; tiles = ceil(W/t) ceil(H/t) for the scene's tile
 * size t, 8 or 4, see prdpt_ctx_create); N doubles if
 * losses_dev is NULL; one int.  Larger requests fail with PRDPT_E_ARG before
 * anything is enqueued.  All calls on one device share that array and each
 * call leaves its contents behind (the work counter is cleared by a kernel at
 * the start of every call): calls that overlap on one device, from different
 * streams or contexts, race and give wrong results, so they must be ordered
 * (the same stream, or events).  PRDPT_E_HIP if the array could not be looked
 * up on the context's device.
 */
#define PRDPT_NOALLOC_SCRATCH_BYTES (16u << 20)
int prdpt_grad_estimate_noalloc(prdpt_scene* scene, const float* ref_dev, const float* theta_dev,
                                const float* sigma_dev, int N, uint64_t seed, int est,
                                double* grad_dev, double* loss_dev, double* losses_dev,
                                double* c_dev);

/*
 * Gradient combination alone (Eq. 10), stream-ordered, for the weights of an
 * estimate made with estimator flags `est`:
 *     grad_dev[j] = scale * (1/P) sum_p c_dev[p][j] (losses_dev[2p] - losses_dev[2p+1])
 * with rows = P pairs, or, with PRDPT_EST_INDEPENDENT in est,
 *     grad_dev[j] = scale * (1/N) sum_i c_dev[i][j] losses_dev[i]
 * with rows = N draws; scale = *scale_dev (device double, NULL means 1).  All
 * pointers device.  1 <= d <= PRDPT_MAX_PARAMS, 1 <= rows <= 2^20, else
 * PRDPT_E_ARG.
 */
int prdpt_combine_async(prdpt_ctx* ctx, int rows, int d, const double* c_dev,
                        const double* losses_dev, const double* scale_dev, double* grad_dev,
                        int est);

/*
 * ---- batched estimation ------------------------------------------------------
 * One request = the arguments of prdpt_grad_estimate for one resident scene of
 * the context.  A batch runs all its valid requests together: one perturbation
 * launch, one persistent render launch whose work-groups take (request,
 * perturbation, run of pixel tiles) items from a device counter, one loss and
 * one combine launch, captured once in a HIP graph and replayed per batch.
 * Every result equals prdpt_grad_estimate of that request alone, bit for bit.
 * A request's scene may have up to PRDPT_BATCH_MAX_PARAMS (= PRDPT_MAX_PARAMS)
 * parameters, as for the single-request calls.
 */
typedef struct {
  prdpt_scene* scene;      /* resident scene of the batch's context */
  const float* ref;        /* device float[H][W][3] */
  const float* theta;      /* host float[d] */
  const float* sigma;      /* host float[d], > 0 */
  int32_t N;               /* even, >= 2 */
  int32_t est;             /* PRDPT_EST_GAUSS / _IS / _IS_PERDIM (antithetic only) */
  uint64_t seed;
  double* grad_out;        /* host double[d] */
  double* loss_out;        /* host double[1] or NULL */
  double* losses_out;      /* host double[N] or NULL */
  int32_t status;          /* out: PRDPT_OK, or the error of this request alone */
} prdpt_request;

/*
 * Run n requests as one batch (synchronous).  Invalid requests get a negative
 * `status` and are skipped without affecting the others; the call itself fails
 * only on context-level errors (allocation, HIP).  The batch runs on a stream
 * the context owns, ordered after work already enqueued on the context stream.
 */
int prdpt_batch_estimate(prdpt_ctx* ctx, prdpt_request* reqs, int n);

/*
 * Launch configuration of the batched form: persistent work-groups per compute
 * unit (0, the default: as many as the compute units hold at once for the
 * batch's largest sphere count), pixel tiles (of the scene's tile size) per
 * work item, and whether to replay a captured graph (1) or launch the kernels
 * directly (0).  The served form takes the context's configuration.
 * Returns PRDPT_E_ARG for blocks_per_cu outside 0..64 or tiles_per_item
 * outside 1..4096.
 */
int prdpt_batch_config(prdpt_ctx* ctx, int blocks_per_cu, int tiles_per_item, int use_graph);

/*
 * Choose blocks_per_cu and tiles_per_item for batches like `reqs` by timing a
 * sweep on them (device time of the graph), and remember the choice per size
 * class (compute units, log2 of camera paths, log2 of requests) in a JSON-lines
 * file at cache_path (nullable: no cache).  A cached size class is applied
 * without a sweep.  Outputs are nullable.
 */
int prdpt_batch_autotune(prdpt_ctx* ctx, prdpt_request* reqs, int n, const char* cache_path,
                         int* best_blocks_per_cu, int* best_tiles_per_item, double* best_ms);

/*
 * ---- serving ------------------------------------------------------------------
 * A request loop for many concurrent inverse-rendering jobs.  Jobs register a
 * scene description and a reference image; their BVHs are built on the host
 * once and kept there.  A server thread forms batch epochs (prdpt_batch_*
 * semantics) from the FIFO of pending requests: a request joins an epoch if its
 * job is resident in HBM or can be admitted within hbm_budget (idle jobs are
 * evicted least recently used first), otherwise it waits for a later epoch.  Up
 * to two epochs run at once on separate streams: requests that arrive while an
 * epoch runs are admitted as slots and memory free up, and overlap it on the
 * device.  Each result equals the request run alone.
 */
typedef struct prdpt_server prdpt_server;

typedef struct {
  size_t hbm_budget;     /* bytes of resident scenes + references (0 = unbounded) */
  int32_t max_batch;     /* requests per epoch (<= 0: 64) */
  int32_t max_inflight;  /* epochs running at once, 1 or 2 (<= 0: 2) */
} prdpt_server_config;

typedef struct {
  int64_t ticket;                 /* from prdpt_server_submit */
  int32_t job;
  int32_t status;                 /* PRDPT_OK, PRDPT_E_CANCELLED, PRDPT_E_ADMISSION, ... */
  double loss;                    /* Q estimate (mean per-image loss) */
  double grad[PRDPT_BATCH_MAX_PARAMS];  /* first d entries valid */
  double t_submit, t_start, t_done;  /* seconds on the server's steady clock */
} prdpt_completion;

typedef struct {
  int64_t submitted, completed, failed, epochs, admissions, evictions, pending, resident_bytes;
  double paths;                   /* camera paths of completed requests */
} prdpt_server_stats;

/* Start the server thread on ctx (which must outlive the server). */
int prdpt_server_start(prdpt_ctx* ctx, const prdpt_server_config* cfg, prdpt_server** out);
/* Register a job: the description is validated and its BVHs built now (host);
 * ref_host is host float[H][W][3], copied.  *job_id receives the job's id.
 * A job's scene has up to PRDPT_BATCH_MAX_PARAMS (= PRDPT_MAX_PARAMS)
 * parameters. */
int prdpt_server_add_job(prdpt_server* sv, const prdpt_scene_desc* desc, const float* ref_host,
                         int* job_id);
/* Queue one gradient estimate of job `job_id` (theta, sigma: host float[d], copied). */
int prdpt_server_submit(prdpt_server* sv, int job_id, const float* theta, const float* sigma, int N,
                        uint64_t seed, int est, int64_t* ticket);
/* As prdpt_server_submit, with a deadline timeout_s seconds after submission
 * (0: none; negative or non-finite: PRDPT_E_ARG).  A request still queued or
 * running when its deadline passes completes at once with PRDPT_E_TIMEOUT (a
 * running one's result is dropped when its epoch ends); the other requests,
 * of its epoch too, are not affected. */
int prdpt_server_submit_deadline(prdpt_server* sv, int job_id, const float* theta,
                                 const float* sigma, int N, uint64_t seed, int est,
                                 double timeout_s, int64_t* ticket);
/* Cancel a queued request (it completes with PRDPT_E_CANCELLED unless already running). */
int prdpt_server_cancel(prdpt_server* sv, int64_t ticket);
/* Take up to max completion records, waiting up to timeout_ms for the first. */
int prdpt_server_poll(prdpt_server* sv, prdpt_completion* out, int max, int timeout_ms, int* n_out);
int prdpt_server_get_stats(prdpt_server* sv, prdpt_server_stats* stats);
/* Finish all queued and running requests (queued requests that can no longer
 * start complete with PRDPT_E_CANCELLED), then release everything.  A job
 * whose upload fails (device memory, the context's budget, HIP) fails its
 * requests with that status instead of holding the queue. */
int prdpt_server_stop(prdpt_server* sv);

/* Wait for all work enqueued on the context's stream. */
int prdpt_ctx_synchronize(prdpt_ctx* ctx);

/*
 * Failure injection for tests of the error paths (process-wide): with
 * after >= 0 the next `after` device or pinned host allocations of the library
 * succeed and every later one fails, so the call that needs it returns
 * PRDPT_E_NOMEM (the server fails that request) and frees what it took;
 * after < 0 turns injection off.  Always PRDPT_OK.
 */
int prdpt_debug_fail_allocations(int64_t after);

/*
 * Measurement hooks.  With timing enabled the context records a pair of HIP
 * events on its stream around every launch of the fused render-and-loss kernel;
 * prdpt_ctx_read_timing waits for them and returns (then clears) the summed
 * kernel time in milliseconds and the number of launches.
 */
int prdpt_ctx_set_timing(prdpt_ctx* ctx, int enable);
int prdpt_ctx_read_timing(prdpt_ctx* ctx, double* total_ms, int64_t* launches);

/*
 * Work of one estimate, measured by an instrumented copy of the render kernel
 * on the same rays: counts[0] BVH nodes fetched, counts[1] triangles tested,
 * counts[2] ray queries (closest-hit and shadow), counts[3] camera paths,
 * counts[4..6] iterations of the node loop, the rounds of triangle tests and
 * iterations of the ray loop executed per wavefront (summed over wavefronts;
 * lane work / (64 x iterations) is each loop's SIMD efficiency), counts[7]
 * lanes idle in ray-loop iterations because their tile has no path left for
 * them (summed over iterations), counts[8] traversal-stack pushes that went to
 * the private part beyond the LDS entries, counts[9] the most stack entries
 * one ray held at once.  counts: host uint64_t[10].  Synchronous.
 */
int prdpt_traversal_counts(prdpt_scene* scene, const float* theta, const float* sigma, int N,
                           uint64_t seed, int est, uint64_t* counts);

/*
 * Achievable-bandwidth probe: copies `bytes` (multiple of 16, 16-byte aligned
 * device buffers) from src to dst `iters` times with a plain streaming kernel on
 * the context's stream and returns the mean milliseconds per copy (each copy
 * reads and writes `bytes`).  Also the reference dispatch for scaling memory
 * counters.  Synchronous.
 */
int prdpt_copy_probe(prdpt_ctx* ctx, const void* src, void* dst, size_t bytes, int iters,
                     double* ms_per_copy);

/*
 * Self-test of the render kernel's arithmetic.  The renderer behind the
 * estimator (Sec. 3.1's black box, made reproducible) rounds every division
 * and square root on its geometric chain correctly, like the reference CPU
 * implementation; the kernel forms 1/x and sqrt(x) from the hardware
 * reciprocal and square root with fused-residual corrections instead of the
 * compiler's longer correctly rounded sequences.  This runs all 2^32
 * binary32 inputs through the three forms (the reciprocal on its domain:
 * +-0, +-inf, NaN and normal |x| <= 2^126; the square root core on its
 * domain: |x| >= 2^-104, +-0, +inf, NaN; the square root for every input)
 * and compares each result with the correctly rounded operation (NaN equals
 * NaN).  mismatches: host uint64_t[3], the three counts in that order (all
 * zero when the forms are exact).  Synchronous; a few milliseconds.
 */
int prdpt_selftest_math(prdpt_ctx* ctx, uint64_t* mismatches);

/*
 * Host-side step of the optimisation loop around the estimator (Sec. 3.3-3.4):
 * linear bandwidth decay sigma_t = sigma0 + (sigma_end - sigma0) t / (T - 1)
 * (the paper's schedule with t normalised to the run length), and one Adam
 * step (Kingma & Ba) on theta with moments m, v (host double[d], updated in
 * place; t counts from 1).
 */
double prdpt_sigma_schedule(double sigma0, double sigma_end, int t, int T);
int prdpt_adam_step(int d, double* theta, const double* grad, double* m, double* v, int t,
                    double lr, double beta1, double beta2, double eps);

#ifdef __cplusplus
}
#endif
#endif /* PRDPT_H */
