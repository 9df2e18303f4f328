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


def _rows(t, rows, name, device=None):
    """(B, ld) of a [rows, B] float32 device tensor with unit stride along B;
    raises before any launch when the tensor cannot be read or written as such."""
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError(f"{name} must be a float32 CUDA tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the guide on {device}")
    if t.dim() != 2 or t.shape[0] != rows or (t.shape[1] > 1 and t.stride(1) != 1):
        raise ValueError(f"{name} must be [{rows}, B] with unit stride along B")
    ld = t.stride(0) if rows > 1 else max(t.shape[1], 1)
    if ld < t.shape[1]:
        raise ValueError(f"{name}: rows overlap (leading dimension {ld} < B = {t.shape[1]})")
    return t.shape[1], ld


def _out_rows(t, rows, B, ld, name, device):
    """Check a caller-supplied [rows][ld] output: the kernels write entries
    0..B-1 of each row at row * ld, so its rows must have the input's stride."""
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or t.device != device:
        raise TypeError(f"{name} must be a float32 tensor on {device}")
    if t.dim() != 2 or t.shape[0] != rows or t.shape[1] < B or (t.shape[1] > 1 and t.stride(1) != 1):
        raise ValueError(f"{name} must be [{rows}, >= {B}] with unit stride along B")
    if rows > 1 and t.stride(0) != ld:
        raise ValueError(f"{name} must have leading dimension {ld} (the input's), not {t.stride(0)}")


def _vec(t, n, name, device):
    """Check a float32 device vector of at least n contiguous elements."""
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or t.device != device:
        raise TypeError(f"{name} must be a float32 tensor on {device}")
    if t.dim() != 1 or t.numel() < n or (t.numel() > 1 and t.stride(0) != 1):
        raise ValueError(f"{name} must be a contiguous 1-D tensor of at least {n} elements")


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

    # -- checkpoints -------------------------------------------------------------
    STATE_KEYS = ("w", "adam_m", "adam_v", "step", "flags")

    def state_dict(self):
        """Host copies of the training state: FP32 master weights, Adam
        moments, the step counter and the flags. Together with the
        configuration they determine every later call bit for bit."""
        torch.cuda.current_stream().synchronize()
        return {k: getattr(self, k).detach().cpu().clone() for k in self.STATE_KEYS}

    def load_state_dict(self, sd):
        """Restore a state_dict() of a guide with the same configuration and
        refresh the kernel-layout copy of the weights."""
        for k in self.STATE_KEYS:
            dst, src = getattr(self, k), sd[k]
            if src.shape != dst.shape or src.dtype != dst.dtype:
                raise ValueError(f"{k}: expected {tuple(dst.shape)} {dst.dtype}, got {tuple(src.shape)} {src.dtype}")
        with torch.no_grad():
            for k in self.STATE_KEYS:
                getattr(self, k).copy_(sd[k])
        self.repack()

    # -- calls -----------------------------------------------------------------
    # Every call checks its tensors (dtype, device, shape, leading dimension,
    # size) and raises before anything is launched: the library receives bare
    # pointers and cannot tell a short or host buffer from a good one.
    @property
    def device(self):
        return self.w.device

    def _rec(self, rec, B):
        n = record_elems(self.n_lobes, B)
        if not isinstance(rec, torch.Tensor) or rec.dtype != torch.float32 or rec.device != self.device:
            raise TypeError(f"rec must be a float32 tensor on {self.device}")
        if not rec.is_contiguous() or rec.numel() < n:
            raise ValueError(f"rec must be contiguous with at least {n} floats (records of {B} vertices)")

    def forward_raw(self, feat, out=None):
        B, ld = _rows(feat, 9, "feat", self.device)
        if out is None:
            out = torch.empty(self.n_out, max(ld, 1), dtype=torch.float32, device=self.device)
        else:
            _out_rows(out, self.n_out, B, ld, "out", self.device)
        check(self.lib.nasg_forward(self._ctx, _ptr(feat), ld, B, _ptr(out), self._stream()))
        return out[:, :B]

    @property
    def n_out(self):
        return 8 * self.n_lobes + (1 if self.selection else 0)

    def query(self, feat, xi, dir_out=None, pdf_out=None, rec_out=None, records=False, sel_out=None):
        """(directions [3, B], pdf [B]) plus the records buffer when requested;
        sel_out (a [B] tensor, selection networks only) receives c."""
        dev = self.device
        B, ld = _rows(feat, 9, "feat", dev)
        Bx, ldx = _rows(xi, 4, "xi", dev)
        if Bx != B or ldx != ld:
            raise ValueError("xi must match feat in B and leading dimension")
        if dir_out is None:
            dir_out = torch.empty(3, max(ld, 1), dtype=torch.float32, device=dev)
        else:
            _out_rows(dir_out, 3, B, ld, "dir_out", dev)
        if pdf_out is None:
            pdf_out = torch.empty(max(B, 1), dtype=torch.float32, device=dev)
        else:
            _vec(pdf_out, B, "pdf_out", dev)
        if records and rec_out is None:
            rec_out = torch.empty(max(record_elems(self.n_lobes, B), 1), dtype=torch.float32, device=dev)
        elif rec_out is not None:
            self._rec(rec_out, B)
        if sel_out is not None:
            if not self.selection:
                raise ValueError("sel_out needs a network with the selection output")
            _vec(sel_out, B, "sel_out", dev)
        check(self.lib.nasg_query(self._ctx, _ptr(feat), _ptr(xi), ld, B, _ptr(dir_out), _ptr(pdf_out),
                                  _ptr(sel_out), _ptr(rec_out), self._stream()))
        if rec_out is not None:
            return dir_out[:, :B], pdf_out[:B], rec_out
        return dir_out[:, :B], pdf_out[:B]

    def pdf(self, rec, dirs, pdf_out=None):
        dev = self.device
        B, ld = _rows(dirs, 3, "dirs", dev)
        self._rec(rec, B)
        if pdf_out is None:
            pdf_out = torch.empty(max(B, 1), dtype=torch.float32, device=dev)
        else:
            _vec(pdf_out, B, "pdf_out", dev)
        check(self.lib.nasg_pdf(self._ctx, _ptr(rec), _ptr(dirs), ld, B, _ptr(pdf_out), self._stream()))
        return pdf_out[:B]

    def pdf_grad(self, rec, dirs, pdf_out=None, grad_out=None):
        """(pdf [B], gradient of log pdf on the sphere [3, B]) at dirs."""
        dev = self.device
        B, ld = _rows(dirs, 3, "dirs", dev)
        self._rec(rec, B)
        if pdf_out is None:
            pdf_out = torch.empty(max(B, 1), dtype=torch.float32, device=dev)
        else:
            _vec(pdf_out, B, "pdf_out", dev)
        if grad_out is None:
            grad_out = torch.empty(3, max(ld, 1), dtype=torch.float32, device=dev)
        else:
            _out_rows(grad_out, 3, B, ld, "grad_out", dev)
        check(self.lib.nasg_pdf_grad(self._ctx, _ptr(rec), _ptr(dirs), ld, B, _ptr(pdf_out), _ptr(grad_out),
                                     self._stream()))
        return pdf_out[:B], grad_out[:, :B]

    def sample(self, rec, xi, dir_out=None, pdf_out=None):
        dev = self.device
        B, ld = _rows(xi, 4, "xi", dev)
        self._rec(rec, B)
        if dir_out is None:
            dir_out = torch.empty(3, max(ld, 1), dtype=torch.float32, device=dev)
        else:
            _out_rows(dir_out, 3, B, ld, "dir_out", dev)
        if pdf_out is None:
            pdf_out = torch.empty(max(B, 1), dtype=torch.float32, device=dev)
        else:
            _vec(pdf_out, B, "pdf_out", dev)
        check(self.lib.nasg_sample(self._ctx, _ptr(rec), _ptr(xi), ld, B, _ptr(dir_out), _ptr(pdf_out),
                                   self._stream()))
        return dir_out[:, :B], pdf_out[:B]

    def _train_args(self, feat, dirs, w, bsdf_pdf):
        dev = self.device
        B, ld = _rows(feat, 9, "feat", dev)
        Bd, ldd = _rows(dirs, 3, "dirs", dev)
        if Bd != B or ldd != ld:
            raise ValueError("dirs must match feat in B and leading dimension")
        _vec(w, B, "w", dev)
        if self.selection:
            if bsdf_pdf is None:
                raise ValueError("a selection network trains on the blended loss: bsdf_pdf is required")
            _vec(bsdf_pdf, B, "bsdf_pdf", dev)
        elif bsdf_pdf is not None:
            raise ValueError("bsdf_pdf needs a network with the selection output")
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
    """Weighted NLL of Sec. 4.2 (or, for a selection network, the blended
    loss) with the library's fused backward.

    loss = NasgNLL.apply(guide.w, guide, feat, dirs, w[, bsdf_pdf]). The
    forward re-packs guide.w into the kernels' layout (a torch optimiser may
    have changed it in place since the last call), then runs the fused kernel
    once: loss and weight gradient together, activations recomputed on chip
    and never stored. backward scales that gradient by the upstream one.
    """

    @staticmethod
    def forward(ctx, weights, guide, feat, dirs, w, bsdf_pdf=None):
        if weights.data_ptr() != guide.w.data_ptr():
            raise ValueError("weights must be guide.w")
        guide.repack()
        guide.loss_grad(feat, dirs, w, bsdf_pdf)
        ctx.grad = guide.grad.clone()
        return guide.stats[0].to(torch.float32)

    @staticmethod
    def backward(ctx, gout):
        return gout * ctx.grad, None, None, None, None, None
