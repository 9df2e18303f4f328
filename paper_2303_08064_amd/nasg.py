"""Python binding of the NASG guiding library (include/nasg.h).

PyTorch provides device memory and streams; every step of the path runs in
the HIP kernels of libnasg.so. Vertex arrays are float32 CUDA tensors laid
out as [rows, B] with unit stride along B (the leading dimension is the row
stride), e.g. features [9, B], uniforms [4, B], directions [3, B].
"""

import ctypes

import torch

from . import _lib
from ._lib import Config, State, check, load

PRECISIONS = {"f32": _lib.NASG_F32, "fp32": _lib.NASG_F32, "bf16": _lib.NASG_BF16}
REC_TILE = 64


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _rows(t, rows, name):
    if t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError(f"{name} must be a float32 CUDA tensor")
    if t.dim() != 2 or t.shape[0] != rows or t.stride(1) != 1:
        raise ValueError(f"{name} must be [{rows}, B] with unit stride along B")
    return t.shape[1], t.stride(0)


def record_elems(n_lobes, B):
    """Floats in a decoded-record buffer for B vertices: tiles of 64 vertices."""
    return ((B + REC_TILE - 1) // REC_TILE) * 9 * n_lobes * REC_TILE


class NasgGuide:
    """Device state of one guiding network plus its context in libnasg.so.

    weights: flat float32 canonical weights (W_0 [hidden][10] or, encoded,
    [hidden][64], W_1..W_{n-1} [hidden][hidden], W_L [8K (+1)][hidden], each
    row-major), e.g. from synth.flat_weights(synth.init_weights(...)).
    selection: the network has the selection-probability output and trains
    on the blended loss with fraction mis_fraction (Sec. 4.2).
    isotropic: a = 0 lobes (normalised spherical Gaussians), for comparisons.
    encoded: W_0 reads the encoded input of Tab. "encoding" (one-blob bins of
    the position, omega_o, n, the one), computed on the device from the same
    9 raw features.
    """

    def __init__(self, weights, hidden=64, n_hidden=4, n_lobes=16, precision="bf16", eps=0.0,
                 lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-8, max_batch=1 << 18, device="cuda",
                 selection=False, mis_fraction=0.2, isotropic=False, encoded=False):
        self.lib = load()
        self.cfg = Config(hidden, n_hidden, n_lobes, PRECISIONS[precision], eps, lr, beta1, beta2,
                          adam_eps, max_batch, int(bool(selection)), mis_fraction, int(bool(isotropic)),
                          int(bool(encoded)))
        self.selection = bool(selection)
        self.encoded = bool(encoded)
        self.n_lobes = n_lobes
        self.hidden = hidden
        self.n_hidden = n_hidden
        self.precision = precision
        nw = self.lib.nasg_num_weights(ctypes.byref(self.cfg))
        pb = self.lib.nasg_packed_bytes(ctypes.byref(self.cfg))
        wb = self.lib.nasg_workspace_bytes(ctypes.byref(self.cfg))
        if pb == 0 or wb == 0:
            raise _lib.NasgError(_lib.NASG_E_ARG, "unsupported configuration")
        w = torch.as_tensor(weights, dtype=torch.float32).reshape(-1)
        if w.numel() != nw:
            raise ValueError(f"expected {nw} weights, got {w.numel()}")
        dev = torch.device(device)
        self.w = w.to(dev).contiguous().clone()
        self.grad = torch.zeros(nw, dtype=torch.float32, device=dev)
        self.adam_m = torch.zeros(nw, dtype=torch.float32, device=dev)
        self.adam_v = torch.zeros(nw, dtype=torch.float32, device=dev)
        self.wpack = torch.zeros(pb, dtype=torch.uint8, device=dev)
        self.step = torch.zeros(1, dtype=torch.int64, device=dev)
        self.flags = torch.zeros(1, dtype=torch.int32, device=dev)
        self.stats = torch.zeros(4, dtype=torch.float64, device=dev)
        self.workspace = torch.zeros(wb, dtype=torch.uint8, device=dev)
        self._state = State(*[t.data_ptr() for t in (self.w, self.grad, self.adam_m, self.adam_v, self.wpack,
                                                      self.step, self.flags, self.stats, self.workspace)])
        torch.cuda.synchronize(dev)
        self._ctx = ctypes.c_void_p()
        check(self.lib.nasg_create(ctypes.byref(self.cfg), ctypes.byref(self._state), ctypes.byref(self._ctx)))

    # -- plumbing ------------------------------------------------------------
    @staticmethod
    def _stream():
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self.lib.nasg_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_weights(self):
        return self.w.numel()

    def repack(self):
        """Refresh the kernel-layout weights after writing self.w directly."""
        check(self.lib.nasg_pack(self._ctx, self._stream()))

    # -- calls -----------------------------------------------------------------
    def forward_raw(self, feat, out=None):
        B, ld = _rows(feat, 9, "feat")
        if out is None:
            out = torch.empty(self.n_out, max(ld, 1), dtype=torch.float32, device=feat.device)
        check(self.lib.nasg_forward(self._ctx, _ptr(feat), ld, B, _ptr(out), self._stream()))
        return out[:, :B]

    @property
    def n_out(self):
        return 8 * self.n_lobes + (1 if self.selection else 0)

    def query(self, feat, xi, dir_out=None, pdf_out=None, rec_out=None, records=False, sel_out=None):
        """(directions [3, B], pdf [B]) plus the records buffer when requested;
        sel_out (a [B] tensor, selection networks only) receives c."""
        B, ld = _rows(feat, 9, "feat")
        Bx, ldx = _rows(xi, 4, "xi")
        if Bx != B or ldx != ld:
            raise ValueError("xi must match feat in B and leading dimension")
        dev = feat.device
        if dir_out is None:
            dir_out = torch.empty(3, max(ld, 1), dtype=torch.float32, device=dev)
        if pdf_out is None:
            pdf_out = torch.empty(max(B, 1), dtype=torch.float32, device=dev)
        if records and rec_out is None:
            rec_out = torch.empty(max(record_elems(self.n_lobes, B), 1), dtype=torch.float32, device=dev)
        if sel_out is not None and (sel_out.dtype != torch.float32 or sel_out.numel() < B):
            raise ValueError("sel_out must be a float32 tensor of at least B elements")
        check(self.lib.nasg_query(self._ctx, _ptr(feat), _ptr(xi), ld, B, _ptr(dir_out), _ptr(pdf_out),
                                  _ptr(sel_out), _ptr(rec_out), self._stream()))
        if rec_out is not None:
            return dir_out[:, :B], pdf_out[:B], rec_out
        return dir_out[:, :B], pdf_out[:B]

    def pdf(self, rec, dirs, pdf_out=None):
        B, ld = _rows(dirs, 3, "dirs")
        if pdf_out is None:
            pdf_out = torch.empty(max(B, 1), dtype=torch.float32, device=dirs.device)
        check(self.lib.nasg_pdf(self._ctx, _ptr(rec), _ptr(dirs), ld, B, _ptr(pdf_out), self._stream()))
        return pdf_out[:B]

    def pdf_grad(self, rec, dirs, pdf_out=None, grad_out=None):
        """(pdf [B], gradient of log pdf on the sphere [3, B]) at dirs."""
        B, ld = _rows(dirs, 3, "dirs")
        dev = dirs.device
        if pdf_out is None:
            pdf_out = torch.empty(max(B, 1), dtype=torch.float32, device=dev)
        if grad_out is None:
            grad_out = torch.empty(3, max(ld, 1), dtype=torch.float32, device=dev)
        check(self.lib.nasg_pdf_grad(self._ctx, _ptr(rec), _ptr(dirs), ld, B, _ptr(pdf_out), _ptr(grad_out),
                                     self._stream()))
        return pdf_out[:B], grad_out[:, :B]

    def sample(self, rec, xi, dir_out=None, pdf_out=None):
        B, ld = _rows(xi, 4, "xi")
        dev = xi.device
        if dir_out is None:
            dir_out = torch.empty(3, max(ld, 1), dtype=torch.float32, device=dev)
        if pdf_out is None:
            pdf_out = torch.empty(max(B, 1), dtype=torch.float32, device=dev)
        check(self.lib.nasg_sample(self._ctx, _ptr(rec), _ptr(xi), ld, B, _ptr(dir_out), _ptr(pdf_out),
                                   self._stream()))
        return dir_out[:, :B], pdf_out[:B]

    def _train_args(self, feat, dirs, w, bsdf_pdf):
        B, ld = _rows(feat, 9, "feat")
        Bd, ldd = _rows(dirs, 3, "dirs")
        if Bd != B or ldd != ld:
            raise ValueError("dirs must match feat in B and leading dimension")
        for t, name in ((w, "w"), (bsdf_pdf, "bsdf_pdf")):
            if t is None:
                continue
            if t.dtype != torch.float32 or t.dim() != 1 or t.shape[0] < B or t.stride(0) != 1:
                raise ValueError(f"{name} must be a contiguous float32 [B] tensor")
        return B, ld

    def loss_grad(self, feat, dirs, w, bsdf_pdf=None):
        """Writes self.grad and self.stats (loss, sum w, -, sum w*(-log term)).
        bsdf_pdf: p_fs at dirs, for selection networks (the blended loss)."""
        B, ld = self._train_args(feat, dirs, w, bsdf_pdf)
        check(self.lib.nasg_loss_grad(self._ctx, _ptr(feat), _ptr(dirs), _ptr(w), _ptr(bsdf_pdf), ld, B,
                                      self._stream()))

    def adam_step(self):
        check(self.lib.nasg_adam_step(self._ctx, self._stream()))

    def train_step(self, feat, dirs, w, bsdf_pdf=None):
        B, ld = self._train_args(feat, dirs, w, bsdf_pdf)
        check(self.lib.nasg_train_step(self._ctx, _ptr(feat), _ptr(dirs), _ptr(w), _ptr(bsdf_pdf), ld, B,
                                       self._stream()))

    # -- views -----------------------------------------------------------------
    def layer_shapes(self):
        s = [(self.hidden, 64 if self.encoded else 10)] + [(self.hidden, self.hidden)] * (self.n_hidden - 1)
        return s + [(self.n_out, self.hidden)]

    def split(self, flat):
        """Flat canonical vector -> list of [out, in] views."""
        out, off = [], 0
        for (o, i) in self.layer_shapes():
            out.append(flat[off:off + o * i].view(o, i))
            off += o * i
        return out


def blend_ramp(frames_done, M=4, B=64):
    """The blend ramp b of Sec. 5 (nasg_blend_ramp)."""
    return float(load().nasg_blend_ramp(int(frames_done), int(M), int(B)))


class NasgNLL(torch.autograd.Function):
    """Weighted NLL of Sec. 4.2 with the library's fused backward.

    loss = NasgNLL.apply(guide.w, guide, feat, dirs, w). The forward runs the
    fused kernel once (loss and weight gradient together, activations
    recomputed on chip and never stored); backward scales that gradient.
    """

    @staticmethod
    def forward(ctx, weights, guide, feat, dirs, w):
        if weights.data_ptr() != guide.w.data_ptr():
            raise ValueError("weights must be guide.w")
        guide.loss_grad(feat, dirs, w)
        ctx.grad = guide.grad.clone()
        return guide.stats[0].to(torch.float32)

    @staticmethod
    def backward(ctx, gout):
        return gout * ctx.grad, None, None, None, None
