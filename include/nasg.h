/*
 * nasg.h -- C ABI of the MI355X (gfx950) NASG path-guiding hot path.
 *
 * Method: "Online Neural Path Guiding with Normalized Anisotropic Spherical
 * Gaussians" (arXiv 2303.08064). A bias-free MLP (Sec. 4.1) maps a path
 * vertex's features (position, outgoing direction, normal) to K NASG lobes
 * (Sec. 3.2, Tab. "decoding"); the normalised mixture (Sec. 3.1) is evaluated
 * in closed form (eq. "K for NASG") and sampled directly (App. C); the MLP is
 * trained online on the weighted negative log-likelihood of sampled
 * directions (Sec. 4.2) with Adam (Sec. 5).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every array argument is a DEVICE pointer owned by the caller. The library
 *   never allocates, frees or retains device memory beyond what the caller
 *   passes in (apart from the fixed scratch array of
 *   nasg_train_step_noalloc); it never synchronises the host.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Every compute call is asynchronous on that stream.
 * - Vertex arrays are structure-of-arrays with leading dimension `ld`
 *   (elements): row r of an [R][ld] array starts at ptr + r*ld, and entries
 *   0..B-1 of each row are used. Requires ld >= B.
 * - Float arrays must be 4-byte aligned.
 * - Errors are reported by return value and never abort: on any status other
 *   than NASG_OK nothing was launched and nasg_last_error() (thread-local)
 *   describes the problem. B == 0 is valid and launches nothing.
 * - Numerical events on the device (NaN/Inf inputs) are not errors: they
 *   propagate to the outputs, and nasg_adam_step skips the update (see below).
 */
#ifndef NASG_H
#define NASG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NASG_OK = 0,
  NASG_E_ARG = 1,    /* null pointer, or a config value outside the supported set */
  NASG_E_SHAPE = 2,  /* B < 0, ld < B, B > max_batch (training calls) */
  NASG_E_ALIGN = 3,  /* misaligned pointer */
  NASG_E_HIP = 4     /* HIP runtime or launch error (message in nasg_last_error) */
} nasg_status;

enum { NASG_F32 = 0, NASG_BF16 = 1 };

/* Network and optimiser configuration.
 * Layers: W_0 is [hidden][10] (9 features + the constant-one input that
 * stands in for the bias, footnote of Sec. 4.1), or [hidden][64] with the
 * encoded input (see `encoding`), then n_hidden-1 matrices [hidden][hidden],
 * then the output W_L [8*n_lobes + selection][hidden]. ReLU between layers,
 * none after the last (Sec. 4.1).
 * Compiled networks: hidden 64 with n_lobes 4, 8 or 16 (raw features, with or
 * without the selection output); hidden 128 with n_lobes 32 (raw features, no
 * selection output); each in FP32 or BF16; and the paper's default network
 * (Sec. 4.1, Sec. 6): hidden 128, n_lobes 8, the selection output and the
 * encoded input, in FP32 or BF16. Hidden-128 networks have n_hidden = 4. */
typedef struct {
  int32_t hidden;      /* 64 or 128 (see the compiled networks above) */
  int32_t n_hidden;    /* number of hidden layers, 1..4 */
  int32_t n_lobes;     /* K: 4, 8, 16 or 32 */
  int32_t precision;   /* NASG_F32: FP32 MFMA; NASG_BF16: BF16 operands, FP32
                          accumulation. NASG math is FP32 in both. */
  float eps;           /* NASG continuity parameter epsilon >= 0 (App. A); 0 = Sec. 3.2 */
  float lr, beta1, beta2, adam_eps;   /* Adam (Sec. 5; Kingma and Ba) */
  int64_t max_batch;   /* largest B accepted by training calls */
  int32_t selection;   /* 1: one more output, the selection probability c = sigmoid(o[8K])
                          (Sec. 4.1, Tab. "decoding"), and training on the blended loss
                          e KL(p||q_hat) + (1-e) KL(p||q), q_hat = c q + (1-c) p_fs
                          (Sec. 4.2); the hidden-64 networks and the paper's default network.
                          0: 8K outputs, NLL of q. */
  float mis_fraction;  /* e of the blended loss, in [0, 1] (the paper uses 0.2) */
  int32_t isotropic;   /* 1: isotropic lobes, a = 0 (normalised spherical Gaussians / vMF, the
                          comparison model of Sec. 6); the a outputs are ignored and get zero
                          gradient. 0: NASG lobes. */
  int32_t encoding;    /* 1: W_0 reads the encoded input of Tab. "encoding", computed on the device
                          from the same 9 raw features: 19 one-blob bins per position coordinate
                          (bin b of coordinate s holds exp(-(19 s - b - 1/2)^2 / 2), a Gaussian of
                          standard deviation 1/19 at the bin centre; s is the position in the
                          scene's bounding box, [0, 1]), then omega_o, n and the constant one: 64
                          inputs. 0: the 9 raw features and the one. */
} nasg_config;

/* Device state, allocated by the caller with the sizes given below.
 * Canonical weight layout: W_0, W_1, ..., W_L concatenated, each row-major
 * [out][in]. Raw output row order of W_L (reading; the paper does not fix it):
 * row p*K + k is parameter p of lobe k, p = 0..7 meaning cos theta, sin phi,
 * cos phi, sin tau, cos tau, log lambda, log a, mixture logit; with the
 * selection output, row 8K is its logit. */
typedef struct {
  float* w;            /* [nasg_num_weights] FP32 master weights (canonical)      */
  float* grad;         /* [nasg_num_weights] dL/dw written by nasg_loss_grad      */
  float* adam_m;       /* [nasg_num_weights] Adam first moment, zero-initialised   */
  float* adam_v;       /* [nasg_num_weights] Adam second moment, zero-initialised  */
  void* wpack;         /* [nasg_packed_bytes] kernel-layout copy of w (16-B aligned) */
  int64_t* step;       /* [1] Adam updates taken so far                            */
  uint32_t* flags;     /* [1] bit 0: the last Adam step was skipped (non-finite)   */
  double* stats;       /* [4] loss L, sum of w, gradient 2-norm, sum of w*(-log term),
                          the log term being log q, or e log q_hat + (1-e) log q */
  void* workspace;     /* [nasg_workspace_bytes] scratch (16-B aligned)            */
} nasg_state;

typedef struct nasg_ctx nasg_ctx;

size_t nasg_num_weights(const nasg_config* cfg);
size_t nasg_packed_bytes(const nasg_config* cfg);
size_t nasg_workspace_bytes(const nasg_config* cfg);

/* Validate cfg and state, bind them to a new host-side context on the
 * current device, and pack state->w into state->wpack on the default stream
 * (synchronised before returning). It also looks up, once per device, the
 * device address of nasg_train_step_noalloc's scratch array. The workspace
 * needs no initialisation. The context is not thread-safe. */
nasg_status nasg_create(const nasg_config* cfg, const nasg_state* state, nasg_ctx** out);
void nasg_destroy(nasg_ctx* ctx);
const char* nasg_last_error(void);

/* Re-pack state->w into state->wpack after the caller changed w directly. */
nasg_status nasg_pack(nasg_ctx* ctx, void* stream);

/* MLP forward only: raw outputs [8K + selection][ld] in canonical row order (Sec. 4.1). */
nasg_status nasg_forward(nasg_ctx* ctx, const float* feat, int64_t ld, int64_t B,
                         float* raw_out, void* stream);

/* Guiding query: fwd + decode + sample + pdf, fused.
 *   feat    [9][ld]  position (3), outgoing direction (3), normal (3)
 *   xi      [4][ld]  uniforms in [0,1): xi_sel picks the lobe by inverse CDF over
 *                    the mixture weights (smallest k with xi_sel < A_0+..+A_k);
 *                    (xi0, xi1) map linearly to (s, rho) and xi2 > 1/2 picks the
 *                    eastern map of App. C
 *   dir_out [3][ld]  sampled unit direction
 *   pdf_out [B]      mixture pdf at dir_out, per steradian (Sec. 3.1)
 *   sel_out [B]      optional (NULL = not written; requires selection = 1): the
 *                    selection probability c. A renderer samples the learned
 *                    distribution with probability b c (b from nasg_blend_ramp)
 *                    and the BSDF otherwise; its MIS pdf is b c q + (1 - b c) p_fs.
 *   rec_out          optional (NULL = not written): decoded lobe records in the
 *                    layout described at nasg_pdf. */
nasg_status nasg_query(nasg_ctx* ctx, const float* feat, const float* xi, int64_t ld, int64_t B,
                       float* dir_out, float* pdf_out, float* sel_out, float* rec_out, void* stream);

/* Mixture pdf at caller directions from decoded records (Sec. 3.1, eq. NASG,
 * eq. "K for NASG"): the pdf a renderer needs for MIS against light samples.
 *   rec  decoded records, tiles of 64 vertices: [ceil(B/64)][9][K][64] floats;
 *        entry (v, p, k) at ((v/64)*9 + p)*K*64 + k*64 + v%64, p = 0..8 meaning
 *        z.x, z.y, z.z, x.x, x.y, x.z, lambda, a, log(A_k / K_k)
 *   dir  [3][ld] directions (normalised inside)
 *   pdf_out [B] */
nasg_status nasg_pdf(nasg_ctx* ctx, const float* rec, const float* dir, int64_t ld, int64_t B,
                     float* pdf_out, void* stream);

/* Mixture pdf and the gradient of log D with respect to the direction, from
 * decoded records (eq. NASG; App. A when eps > 0), for downstream uses such as
 * MIS weights over a solid-angle neighbourhood or denoising:
 *   dir      [3][ld] directions (normalised inside)
 *   pdf_out  [B]
 *   grad_out [3][ld] the gradient on the sphere at dir/|dir| (tangent to it;
 *            the Euclidean gradient of log D(d/|d|) at a unit d). */
nasg_status nasg_pdf_grad(nasg_ctx* ctx, const float* rec, const float* dir, int64_t ld, int64_t B,
                          float* pdf_out, float* grad_out, void* stream);

/* Direct sampling from decoded records (App. C), with the inverse-CDF lobe
 * choice of nasg_query; writes the direction and the mixture pdf there. */
nasg_status nasg_sample(nasg_ctx* ctx, const float* rec, const float* xi, int64_t ld, int64_t B,
                        float* dir_out, float* pdf_out, void* stream);

/* Weighted NLL and its gradient (Sec. 4.2): L = (1/B) sum_j w_j (-log q(dir_j|feat_j)),
 * or with selection = 1 the blended loss
 * L = (1/B) sum_j w_j (-(e log q_hat_j + (1 - e) log q_j)), q_hat = c q + (1 - c) p_fs.
 *   feat [9][ld], dir [3][ld] (normalised inside), w [B] = p / q_hat per sample
 *   (q_hat: the density the sample was drawn from)
 *   bsdf_pdf [B] p_fs at dir, required with selection = 1 and NULL otherwise.
 * Writes state->grad (canonical layout) and state->stats[0..1,3]. Activations
 * are recomputed, never stored. Requires 0 < B <= max_batch. */
nasg_status nasg_loss_grad(nasg_ctx* ctx, const float* feat, const float* dir, const float* w,
                           const float* bsdf_pdf, int64_t ld, int64_t B, void* stream);

/* One Adam update of state->w from state->grad (bias-corrected, no decay), with
 * state->wpack refreshed in the same kernel. Skipped, with flags bit 0 set and
 * step unchanged, when the loss or the gradient norm is not finite.
 * Must follow nasg_loss_grad on the same stream. */
nasg_status nasg_adam_step(nasg_ctx* ctx, void* stream);

/* nasg_loss_grad followed by nasg_adam_step. */
nasg_status nasg_train_step(nasg_ctx* ctx, const float* feat, const float* dir, const float* w,
                            const float* bsdf_pdf, int64_t ld, int64_t B, void* stream);

/* nasg_train_step without the caller's workspace, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid allocation). The same kernels and results as
 * nasg_train_step, bit for bit; the step's scratch (per-workgroup gradient
 * partials, loss and gradient-norm partials, the step snapshot) lives in a
 * 24 MiB array that the library holds on each GPU it runs on until the
 * process ends (its address is looked up once per device by nasg_create).
 * Every call on a GPU shares that GPU's array and needs none of its
 * previous contents: calls that overlap on one GPU (on different streams, or
 * with nasg_train_step_noalloc of another context) race and must be
 * ordered by the caller. The state arrays (weights, moments, grad, flags,
 * stats) are still the context's.
 * Serves hidden-64 networks (NASG_E_ARG for hidden 128); NASG_E_SHAPE if the
 * step's workspace would exceed the scratch (not the case for any compiled
 * hidden-64 network); NASG_E_ARG if the current device is not the context's.
 * Arguments and the other errors as nasg_train_step. */
nasg_status nasg_train_step_noalloc(nasg_ctx* ctx, const float* feat, const float* dir, const float* w,
                                    const float* bsdf_pdf, int64_t ld, int64_t B, void* stream);

/* The blend ramp b of Sec. 5 (host only): 0 at the start, raised by 1/B after
 * every M rendered images, capped at 1 (the paper uses M = 4, B = 64).
 * Returns 0 for frames_done <= 0 or non-positive M, B. */
float nasg_blend_ramp(int64_t frames_done, int32_t M, int32_t B);

#ifdef __cplusplus
}
#endif

#endif /* NASG_H */
