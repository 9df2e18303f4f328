// C ABI of include/nasg.h: host-side validation, workspace carving and
// kernel launches. No call allocates device memory or synchronises, except
// nasg_create, which packs the weights and waits for that to finish.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>

#include "kernels.hpp"
#include "nasg.h"

using namespace nasg;

namespace {

thread_local std::string g_err;

nasg_status fail(nasg_status s, const char* fn, const char* what) {
  g_err = std::string(fn) + ": " + what;
  return s;
}

nasg_status hip_fail(const char* fn, hipError_t e) {
  g_err = std::string(fn) + ": HIP error: " + hipGetErrorString(e);
  return NASG_E_HIP;
}

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// hidden-64 networks: any (K, precision) of the list, with or without the
// selection output, on the raw features
bool small_compiled(const nasg_config* c) {
#define NASG_CASE(h, k, p) \
  if (c->hidden == h && c->n_lobes == k && c->precision == p && c->encoding == 0) return true;
  NASG_FOR_EACH_NET(NASG_CASE)
#undef NASG_CASE
  return false;
}

// hidden-128 networks: exactly the listed variants
bool large_compiled(const nasg_config* c) {
#define NASG_CASE(h, k, p, s, e)                                                                     \
  if (c->hidden == h && c->n_lobes == k && c->precision == p && c->selection == s && c->encoding == e) \
    return true;
  NASG_FOR_EACH_LARGE_NET(NASG_CASE)
#undef NASG_CASE
  return false;
}

bool is_large(const nasg_config* c) { return c->hidden == 128; }

NetDims dims_of(const nasg_config* c) {
  return NetDims{c->hidden, c->n_hidden, c->n_lobes, c->selection, c->encoding};
}

const char* config_error(const nasg_config* c) {
  if (c == nullptr) return "config is NULL";
  if (c->n_hidden < 1 || c->n_hidden > 4) return "n_hidden must be in 1..4";
  if (c->precision != NASG_F32 && c->precision != NASG_BF16) return "precision must be NASG_F32 or NASG_BF16";
  if (c->selection != 0 && c->selection != 1) return "selection must be 0 or 1";
  if (c->encoding != 0 && c->encoding != 1) return "encoding must be 0 or 1";
  if (!(is_large(c) ? large_compiled(c) : small_compiled(c)))
    return "unsupported network; compiled: hidden 64 with n_lobes 4, 8 or 16 on the raw features, with or "
           "without the selection output; hidden 128 with n_lobes 32 on the raw features without it; each in "
           "FP32 or BF16; and the paper's network, hidden 128 with n_lobes 8, the selection output and the "
           "encoded input, in FP32 or BF16";
  if (is_large(c) && c->n_hidden != 4) return "hidden 128 networks are compiled for n_hidden = 4";
  if (!(c->mis_fraction >= 0.0f && c->mis_fraction <= 1.0f)) return "mis_fraction must be in [0, 1]";
  if (c->isotropic != 0 && c->isotropic != 1) return "isotropic must be 0 or 1";
  if (!(c->eps >= 0.0f) || !isfinite(c->eps)) return "eps must be finite and >= 0";
  if (!(c->lr > 0.0f) || !isfinite(c->lr)) return "lr must be finite and > 0";
  if (!(c->beta1 >= 0.0f && c->beta1 < 1.0f) || !(c->beta2 >= 0.0f && c->beta2 < 1.0f))
    return "beta1 and beta2 must be in [0, 1)";
  if (!(c->adam_eps > 0.0f) || !isfinite(c->adam_eps)) return "adam_eps must be finite and > 0";
  if (c->max_batch < 0) return "max_batch must be >= 0";
  if (dims_of(c).num_weights() % 4 != 0) return "the weight count must be a multiple of 4";
  return nullptr;
}

struct Workspace {
  size_t partial, loss_partial, norm_partial, step_snapshot, dout, total;
};

Workspace carve(const nasg_config* c) {
  const int64_t nw = dims_of(c).num_weights();
  Workspace w;
  size_t off = 0;
  w.partial = off;
  off = align_up(off + (size_t)kMaxTrainWG * nw * sizeof(float));
  w.loss_partial = off;
  off = align_up(off + (size_t)2 * kMaxTrainWG * 2 * sizeof(double));
  w.norm_partial = off;
  off = align_up(off + (size_t)reduce_blocks(nw) * sizeof(double));
  w.step_snapshot = off;
  off = align_up(off + sizeof(int64_t));
  w.dout = off;
  if (is_large(c)) {
    // dL/d(raw outputs) of every sample of a training batch, BF16 or FP32 as the network
    off = align_up(off + large_dout_bytes(c->max_batch, c->n_lobes, c->selection, c->precision));
  }
  w.total = off;
  return w;
}

size_t packed_elems(const nasg_config* c) {
  NetDims d = dims_of(c);
  return c->precision == NASG_BF16 ? (size_t)Bf16Layout{d}.total_elems() : (size_t)F32Layout{d}.total_elems();
}

size_t packed_bytes_of(const nasg_config* c) {
  return packed_elems(c) * (c->precision == NASG_BF16 ? 2 : 4);
}

// LDS bytes the query kernel copies: the forward part of the packed weights
size_t query_lds_bytes(const nasg_config* c) {
  NetDims d = dims_of(c);
  if (c->precision == NASG_BF16) return (size_t)Bf16Layout{d}.fwd_elems() * 2;
  return (size_t)F32Layout{d}.total_elems() * 4;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace

struct nasg_ctx {
  nasg_config cfg;
  nasg_state st;
  NetDims d;
  Workspace ws;
  int num_cus;
  int device;
  int q_per_cu[2];   // resident query kernel's workgroups per CU (query, raw forward)
};

namespace {

// ---- scratch of the entry point without allocation ----
// nasg_train_step_noalloc keeps the training step's workspace (per-workgroup
// gradient partials, loss and gradient-norm partials, the step snapshot) in
// this file-scope device array instead of the caller's workspace. Hidden-64
// networks need at most 256 partials of 21184 weights (K = 16 with the
// selection output): 21.7 MB of the 24 MiB. In host code `scratch` only
// names the symbol; its device address, one per GPU, comes from
// hipGetSymbolAddress (scratch_ptr), which every use goes through.
constexpr size_t kScratchBytes = (size_t)24 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's address on `dev` (the current device), looked up once.
hipError_t scratch_ptr(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

size_t nasg_num_weights(const nasg_config* cfg) {
  if (cfg == nullptr) return 0;
  return (size_t)dims_of(cfg).num_weights();
}

size_t nasg_packed_bytes(const nasg_config* cfg) {
  if (config_error(cfg) != nullptr) return 0;
  return packed_bytes_of(cfg);
}

size_t nasg_workspace_bytes(const nasg_config* cfg) {
  if (config_error(cfg) != nullptr) return 0;
  return carve(cfg).total;
}

const char* nasg_last_error(void) { return g_err.c_str(); }

nasg_status nasg_create(const nasg_config* cfg, const nasg_state* st, nasg_ctx** out) {
  static const char* fn = "nasg_create";
  if (out == nullptr) return fail(NASG_E_ARG, fn, "out is NULL");
  *out = nullptr;
  if (const char* e = config_error(cfg)) return fail(NASG_E_ARG, fn, e);
  if (st == nullptr) return fail(NASG_E_ARG, fn, "state is NULL");
  if (!st->w || !st->grad || !st->adam_m || !st->adam_v || !st->wpack || !st->step || !st->flags || !st->stats ||
      !st->workspace)
    return fail(NASG_E_ARG, fn, "a state pointer is NULL");
  if (!aligned(st->w, 4) || !aligned(st->grad, 4) || !aligned(st->adam_m, 4) || !aligned(st->adam_v, 4) ||
      !aligned(st->step, 8) || !aligned(st->flags, 4) || !aligned(st->stats, 8))
    return fail(NASG_E_ALIGN, fn, "state arrays must be naturally aligned");
  if (!aligned(st->wpack, 16) || !aligned(st->workspace, 16))
    return fail(NASG_E_ALIGN, fn, "wpack and workspace must be 16-byte aligned");
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(fn, e);
  void* scr = nullptr;
  e = scratch_ptr(dev, &scr);   // once per device: the allocation-free entry point's scratch
  if (e != hipSuccess) return hip_fail(fn, e);
  nasg_ctx* c = new nasg_ctx;
  c->cfg = *cfg;
  c->st = *st;
  c->d = dims_of(cfg);
  c->ws = carve(cfg);
  c->num_cus = cus > 0 ? cus : 1;
  c->device = dev;
  c->q_per_cu[0] = c->q_per_cu[1] = 1;
  if (query_is_resident(c->d, cfg->precision)) {
    for (int mode = 0; mode < 2 && e == hipSuccess; ++mode)
      e = query_workgroups_per_cu(c->d, cfg->precision, mode, (int)query_lds_bytes(cfg), &c->q_per_cu[mode]);
    if (e != hipSuccess) {
      delete c;
      return hip_fail(fn, e);
    }
  }
  e = launch_pack(st->w, st->wpack, c->d, cfg->precision, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(fn, e);
  }
  *out = c;
  return NASG_OK;
}

void nasg_destroy(nasg_ctx* ctx) { delete ctx; }

nasg_status nasg_pack(nasg_ctx* ctx, void* stream) {
  if (ctx == nullptr) return fail(NASG_E_ARG, "nasg_pack", "ctx is NULL");
  hipError_t e = launch_pack(ctx->st.w, ctx->st.wpack, ctx->d, ctx->cfg.precision, (hipStream_t)stream);
  return e == hipSuccess ? NASG_OK : hip_fail("nasg_pack", e);
}

static nasg_status check_batch(const char* fn, int64_t ld, int64_t B) {
  if (B < 0) return fail(NASG_E_SHAPE, fn, "B < 0");
  if (ld < B) return fail(NASG_E_SHAPE, fn, "ld < B");
  return NASG_OK;
}

static nasg_status check_ptr(const char* fn, const void* p, const char* name) {
  if (p == nullptr) return fail(NASG_E_ARG, fn, (std::string(name) + " is NULL").c_str());
  if (!aligned(p, 4)) return fail(NASG_E_ALIGN, fn, (std::string(name) + " is not 4-byte aligned").c_str());
  return NASG_OK;
}

#define NASG_TRY(x)                      \
  do {                                   \
    nasg_status s_ = (x);                \
    if (s_ != NASG_OK) return s_;        \
  } while (0)

static nasg_status run_query(nasg_ctx* ctx, const char* fn, const float* feat, const float* xi, int64_t ld,
                             int64_t B, float* dir_out, float* pdf_out, float* sel_out, float* rec_out,
                             float* raw_out, int mode, void* stream) {
  if (ctx == nullptr) return fail(NASG_E_ARG, fn, "ctx is NULL");
  NASG_TRY(check_batch(fn, ld, B));
  if (B == 0) return NASG_OK;
  NASG_TRY(check_ptr(fn, feat, "feat"));
  if (mode == 0) {
    NASG_TRY(check_ptr(fn, xi, "xi"));
    NASG_TRY(check_ptr(fn, dir_out, "dir_out"));
    NASG_TRY(check_ptr(fn, pdf_out, "pdf_out"));
    if (rec_out != nullptr && !aligned(rec_out, 4)) return fail(NASG_E_ALIGN, fn, "rec_out is not 4-byte aligned");
    if (sel_out != nullptr) {
      if (ctx->cfg.selection != 1) return fail(NASG_E_ARG, fn, "sel_out needs a network with the selection output");
      if (!aligned(sel_out, 4)) return fail(NASG_E_ALIGN, fn, "sel_out is not 4-byte aligned");
    }
  } else {
    NASG_TRY(check_ptr(fn, raw_out, "raw_out"));
  }
  QueryArgs a;
  a.wpack = ctx->st.wpack;
  a.lds_bytes = (int)query_lds_bytes(&ctx->cfg);
  a.nh = ctx->d.NH;
  a.eps = ctx->cfg.eps;
  a.feat = feat;
  a.xi = xi;
  a.ld = ld;
  a.B = B;
  a.dir_out = dir_out;
  a.pdf_out = pdf_out;
  a.rec_out = rec_out;
  a.raw_out = raw_out;
  a.sel_out = sel_out;
  a.sel = ctx->d.S;
  a.amul = ctx->cfg.isotropic ? 0.0f : 1.0f;
  a.num_cus = ctx->num_cus;
  a.per_cu = ctx->q_per_cu[mode];
  hipError_t e = query_is_resident(ctx->d, ctx->cfg.precision)
                     ? launch_query(a, ctx->d, ctx->cfg.precision, mode, (hipStream_t)stream)
                     : launch_large_query(a, ctx->d, ctx->cfg.precision, mode, (hipStream_t)stream);
  return e == hipSuccess ? NASG_OK : hip_fail(fn, e);
}

nasg_status nasg_forward(nasg_ctx* ctx, const float* feat, int64_t ld, int64_t B, float* raw_out, void* stream) {
  return run_query(ctx, "nasg_forward", feat, nullptr, ld, B, nullptr, nullptr, nullptr, nullptr, raw_out, 1,
                   stream);
}

nasg_status nasg_query(nasg_ctx* ctx, const float* feat, const float* xi, int64_t ld, int64_t B, float* dir_out,
                       float* pdf_out, float* sel_out, float* rec_out, void* stream) {
  return run_query(ctx, "nasg_query", feat, xi, ld, B, dir_out, pdf_out, sel_out, rec_out, nullptr, 0, stream);
}

nasg_status nasg_pdf(nasg_ctx* ctx, const float* rec, const float* dir, int64_t ld, int64_t B, float* pdf_out,
                     void* stream) {
  static const char* fn = "nasg_pdf";
  if (ctx == nullptr) return fail(NASG_E_ARG, fn, "ctx is NULL");
  NASG_TRY(check_batch(fn, ld, B));
  if (B == 0) return NASG_OK;
  NASG_TRY(check_ptr(fn, rec, "rec"));
  NASG_TRY(check_ptr(fn, dir, "dir"));
  NASG_TRY(check_ptr(fn, pdf_out, "pdf_out"));
  RecArgs a{rec, dir, nullptr, ld, B, ctx->cfg.eps, nullptr, pdf_out, nullptr};
  hipError_t e = launch_pdf(a, ctx->d.K, (hipStream_t)stream);
  return e == hipSuccess ? NASG_OK : hip_fail(fn, e);
}

nasg_status nasg_pdf_grad(nasg_ctx* ctx, const float* rec, const float* dir, int64_t ld, int64_t B,
                          float* pdf_out, float* grad_out, void* stream) {
  static const char* fn = "nasg_pdf_grad";
  if (ctx == nullptr) return fail(NASG_E_ARG, fn, "ctx is NULL");
  NASG_TRY(check_batch(fn, ld, B));
  if (B == 0) return NASG_OK;
  NASG_TRY(check_ptr(fn, rec, "rec"));
  NASG_TRY(check_ptr(fn, dir, "dir"));
  NASG_TRY(check_ptr(fn, pdf_out, "pdf_out"));
  NASG_TRY(check_ptr(fn, grad_out, "grad_out"));
  RecArgs a{rec, dir, nullptr, ld, B, ctx->cfg.eps, nullptr, pdf_out, grad_out};
  hipError_t e = launch_pdf_grad(a, ctx->d.K, (hipStream_t)stream);
  return e == hipSuccess ? NASG_OK : hip_fail(fn, e);
}

nasg_status nasg_sample(nasg_ctx* ctx, const float* rec, const float* xi, int64_t ld, int64_t B, float* dir_out,
                        float* pdf_out, void* stream) {
  static const char* fn = "nasg_sample";
  if (ctx == nullptr) return fail(NASG_E_ARG, fn, "ctx is NULL");
  NASG_TRY(check_batch(fn, ld, B));
  if (B == 0) return NASG_OK;
  NASG_TRY(check_ptr(fn, rec, "rec"));
  NASG_TRY(check_ptr(fn, xi, "xi"));
  NASG_TRY(check_ptr(fn, dir_out, "dir_out"));
  NASG_TRY(check_ptr(fn, pdf_out, "pdf_out"));
  RecArgs a{rec, nullptr, xi, ld, B, ctx->cfg.eps, dir_out, pdf_out, nullptr};
  hipError_t e = launch_sample(a, ctx->d.K, (hipStream_t)stream);
  return e == hipSuccess ? NASG_OK : hip_fail(fn, e);
}

// ws: the workspace base (the caller's, or the scratch array's address)
static nasg_status adam_only(nasg_ctx* ctx, const char* fn, unsigned char* ws, void* stream) {
  const nasg_state& s = ctx->st;
  AdamArgs a;
  a.w = s.w;
  a.m = s.adam_m;
  a.v = s.adam_v;
  a.grad = s.grad;
  a.wpack = s.wpack;
  a.step = s.step;
  a.step_snapshot = reinterpret_cast<const int64_t*>(ws + ctx->ws.step_snapshot);
  a.flags = s.flags;
  a.stats = s.stats;
  a.norm_partial = reinterpret_cast<const double*>(ws + ctx->ws.norm_partial);
  a.n_norm = reduce_blocks(ctx->d.num_weights());
  a.n_weights = ctx->d.num_weights();
  a.H = ctx->d.H;
  a.NH = ctx->d.NH;
  a.K = ctx->d.K;
  a.S = ctx->d.S;
  a.E = ctx->d.E;
  a.prec = ctx->cfg.precision;
  a.lr = ctx->cfg.lr;
  a.beta1 = ctx->cfg.beta1;
  a.beta2 = ctx->cfg.beta2;
  a.adam_eps = ctx->cfg.adam_eps;
  hipError_t e = launch_adam(a, (hipStream_t)stream);
  return e == hipSuccess ? NASG_OK : hip_fail(fn, e);
}

// the loss and gradient launches of nasg_loss_grad and nasg_train_step; fn
// names the entry point in error messages
static nasg_status loss_grad(nasg_ctx* ctx, const char* fn, const float* feat, const float* dir, const float* w,
                             const float* bsdf_pdf, int64_t ld, int64_t B, unsigned char* ws, void* stream) {
  if (ctx == nullptr) return fail(NASG_E_ARG, fn, "ctx is NULL");
  NASG_TRY(check_batch(fn, ld, B));
  if (B > ctx->cfg.max_batch) return fail(NASG_E_SHAPE, fn, "B > max_batch");
  if (B == 0) return fail(NASG_E_SHAPE, fn, "B == 0: the mean loss is undefined");
  NASG_TRY(check_ptr(fn, feat, "feat"));
  NASG_TRY(check_ptr(fn, dir, "dir"));
  NASG_TRY(check_ptr(fn, w, "w"));
  if (ctx->cfg.selection == 1) NASG_TRY(check_ptr(fn, bsdf_pdf, "bsdf_pdf"));
  else if (bsdf_pdf != nullptr) return fail(NASG_E_ARG, fn, "bsdf_pdf needs a network with the selection output");
  const nasg_state& s = ctx->st;
  const bool large = is_large(&ctx->cfg);
  const int n_wg = large ? large_train_workgroups(B, ctx->num_cus, ctx->cfg.precision)
                         : train_workgroups(B, ctx->num_cus);
  const int n_loss = large ? large_loss_workgroups(B, ctx->num_cus, ctx->cfg.precision) : n_wg;
  TrainArgs t;
  t.wpack = s.wpack;
  t.lds_bytes = (int)packed_bytes_of(&ctx->cfg);
  t.nh = ctx->d.NH;
  t.eps = ctx->cfg.eps;
  t.feat = feat;
  t.dir = dir;
  t.w = w;
  t.ld = ld;
  t.B = B;
  t.partial = reinterpret_cast<float*>(ws + ctx->ws.partial);
  t.loss_partial = reinterpret_cast<double*>(ws + ctx->ws.loss_partial);
  t.n_weights = ctx->d.num_weights();
  t.num_cus = ctx->num_cus;
  t.sel = ctx->d.S;
  t.bsdf_pdf = bsdf_pdf;
  t.mis_e = ctx->cfg.mis_fraction;
  t.amul = ctx->cfg.isotropic ? 0.0f : 1.0f;
  hipError_t e;
  if (large) {
    LargeTrainArgs la;
    la.wpack = s.wpack;
    la.eps = ctx->cfg.eps;
    la.feat = feat;
    la.dir = dir;
    la.w = w;
    la.bsdf_pdf = bsdf_pdf;
    la.mis_e = ctx->cfg.mis_fraction;
    la.ld = ld;
    la.B = B;
    la.dout = ws + ctx->ws.dout;
    la.partial = t.partial;
    la.loss_partial = t.loss_partial;
    la.n_weights = t.n_weights;
    la.amul = t.amul;
    la.num_cus = ctx->num_cus;
    e = launch_large_train(la, ctx->d, ctx->cfg.precision, n_wg, n_loss, (hipStream_t)stream);
  } else {
    e = launch_train(t, ctx->d.H, ctx->d.K, ctx->cfg.precision, n_wg, (hipStream_t)stream);
  }
  if (e != hipSuccess) return hip_fail(fn, e);
  ReduceArgs r;
  r.partial = t.partial;
  r.loss_partial = t.loss_partial;
  r.n_wg = n_wg;
  r.n_loss = n_loss;
  r.n_weights = t.n_weights;
  r.B = B;
  r.grad = s.grad;
  r.norm_partial = reinterpret_cast<double*>(ws + ctx->ws.norm_partial);
  r.stats = s.stats;
  r.step = s.step;
  r.step_snapshot = reinterpret_cast<int64_t*>(ws + ctx->ws.step_snapshot);
  e = launch_reduce(r, reduce_blocks(t.n_weights), (hipStream_t)stream);
  return e == hipSuccess ? NASG_OK : hip_fail(fn, e);
}

nasg_status nasg_loss_grad(nasg_ctx* ctx, const float* feat, const float* dir, const float* w,
                           const float* bsdf_pdf, int64_t ld, int64_t B, void* stream) {
  if (ctx == nullptr) return fail(NASG_E_ARG, "nasg_loss_grad", "ctx is NULL");
  return loss_grad(ctx, "nasg_loss_grad", feat, dir, w, bsdf_pdf, ld, B,
                   static_cast<unsigned char*>(ctx->st.workspace), stream);
}

nasg_status nasg_adam_step(nasg_ctx* ctx, void* stream) {
  if (ctx == nullptr) return fail(NASG_E_ARG, "nasg_adam_step", "ctx is NULL");
  return adam_only(ctx, "nasg_adam_step", static_cast<unsigned char*>(ctx->st.workspace), stream);
}

nasg_status nasg_train_step(nasg_ctx* ctx, const float* feat, const float* dir, const float* w,
                            const float* bsdf_pdf, int64_t ld, int64_t B, void* stream) {
  if (ctx == nullptr) return fail(NASG_E_ARG, "nasg_train_step", "ctx is NULL");
  unsigned char* ws = static_cast<unsigned char*>(ctx->st.workspace);
  NASG_TRY(loss_grad(ctx, "nasg_train_step", feat, dir, w, bsdf_pdf, ld, B, ws, stream));
  return adam_only(ctx, "nasg_train_step", ws, stream);
}

nasg_status nasg_train_step_noalloc(nasg_ctx* ctx, const float* feat, const float* dir, const float* w,
                                    const float* bsdf_pdf, int64_t ld, int64_t B, void* stream) {
  static const char* fn = "nasg_train_step_noalloc";
  if (ctx == nullptr) return fail(NASG_E_ARG, fn, "ctx is NULL");
  if (is_large(&ctx->cfg)) return fail(NASG_E_ARG, fn, "serves hidden-64 networks only");
  if (ctx->ws.total > kScratchBytes) return fail(NASG_E_SHAPE, fn, "the step's workspace exceeds the 24 MiB scratch");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(fn, e);
  if (dev != ctx->device) return fail(NASG_E_ARG, fn, "the current device is not the one the context was created on");
  void* scr = nullptr;
  e = scratch_ptr(dev, &scr);
  if (e != hipSuccess) return hip_fail(fn, e);
  unsigned char* ws = static_cast<unsigned char*>(scr);
  NASG_TRY(loss_grad(ctx, fn, feat, dir, w, bsdf_pdf, ld, B, ws, stream));
  return adam_only(ctx, fn, ws, stream);
}

float nasg_blend_ramp(int64_t frames_done, int32_t M, int32_t B) {
  if (frames_done <= 0 || M <= 0 || B <= 0) return 0.0f;
  const int64_t steps = frames_done / M;
  return steps >= B ? 1.0f : (float)steps / (float)B;
}

}  // extern "C"
