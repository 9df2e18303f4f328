"""Host-side checks: kernel weight layouts and the C ABI's exports (no GPU)."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nasg.h")
CSRC = os.path.join(ROOT, "paper_2303_08064_amd", "csrc")


def test_weight_layouts_are_bijections(tmp_path):
    exe = tmp_path / "layout_check"
    src = os.path.join(ROOT, "tests", "layout_check.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, src, "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr


def header_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(nasg_[a-z_]+)\s*\(", text)))


def test_header_matches_binding_list():
    from paper_2303_08064_amd import _lib
    assert header_functions() == sorted(_lib.EXPORTED)


@pytest.fixture(scope="module")
def lib():
    from paper_2303_08064_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libnasg.so is not built; run `python -m paper_2303_08064_amd.build`")
    return _lib.load()


def test_library_exports_every_declared_symbol(lib):
    for name in header_functions():
        assert hasattr(lib, name), name


def _cfg(**kw):
    from paper_2303_08064_amd._lib import Config
    base = dict(hidden=64, n_hidden=4, n_lobes=16, precision=1, eps=0.0, lr=1e-3, beta1=0.9,
                beta2=0.999, adam_eps=1e-8, max_batch=1 << 18, selection=0, mis_fraction=0.2, isotropic=0,
                encoding=0)
    base.update(kw)
    return Config(**base)


def test_size_queries(lib):
    c = _cfg()
    assert lib.nasg_num_weights(ctypes.byref(c)) == 21120
    # bf16 fragments: forward 16H + 3H^2 + 8KH, backward 3H^2 + 8KH, 2 bytes each
    assert lib.nasg_packed_bytes(ctypes.byref(c)) == 2 * (1024 + 3 * 4096 + 8192 + 3 * 4096 + 8192)
    c32 = _cfg(precision=0, n_lobes=8)
    assert lib.nasg_num_weights(ctypes.byref(c32)) == 17024
    assert lib.nasg_packed_bytes(ctypes.byref(c32)) == 4 * (64 * 17 + 3 * 64 * 65 + 64 * 65)
    ws = lib.nasg_workspace_bytes(ctypes.byref(c))
    assert ws >= 256 * 21120 * 4
    # unsupported configurations report zero sizes
    assert lib.nasg_packed_bytes(ctypes.byref(_cfg(hidden=48))) == 0
    assert lib.nasg_workspace_bytes(ctypes.byref(_cfg(n_lobes=5))) == 0
    # the large network: 4 hidden layers; its workspace holds the raw-output
    # gradient of a whole batch (512 B per sample at K = 32 in BF16, 1 KiB in FP32)
    big = _cfg(hidden=128, n_lobes=32, max_batch=1 << 12)
    assert lib.nasg_num_weights(ctypes.byref(big)) == 83200
    assert lib.nasg_workspace_bytes(ctypes.byref(big)) >= 256 * 83200 * 4 + (1 << 12) * 512
    big32 = _cfg(hidden=128, n_lobes=32, precision=0, max_batch=1 << 12)
    assert lib.nasg_workspace_bytes(ctypes.byref(big32)) >= 256 * 83200 * 4 + (1 << 12) * 1024
    assert lib.nasg_packed_bytes(ctypes.byref(big32)) == 4 * (128 * 17 + 3 * 128 * 129 + 256 * 129)
    assert lib.nasg_packed_bytes(ctypes.byref(_cfg(hidden=128, n_lobes=32, n_hidden=3))) == 0


def test_create_validates_on_host(lib):
    from paper_2303_08064_amd._lib import State, NASG_E_ARG
    ctx = ctypes.c_void_p()
    st = State()
    assert lib.nasg_create(ctypes.byref(_cfg()), ctypes.byref(st), ctypes.byref(ctx)) == NASG_E_ARG
    assert b"NULL" in lib.nasg_last_error()
    assert lib.nasg_create(ctypes.byref(_cfg(n_hidden=9)), ctypes.byref(st), ctypes.byref(ctx)) == NASG_E_ARG
    assert b"n_hidden" in lib.nasg_last_error()
    assert lib.nasg_create(ctypes.byref(_cfg(lr=-1.0)), ctypes.byref(st), ctypes.byref(ctx)) == NASG_E_ARG
    assert lib.nasg_query(None, None, None, 0, 0, None, None, None, None, None) == NASG_E_ARG
    # the selection output: hidden-64 networks only, mis_fraction in [0, 1]
    assert lib.nasg_create(ctypes.byref(_cfg(hidden=128, n_lobes=32, selection=1)), ctypes.byref(st),
                           ctypes.byref(ctx)) == NASG_E_ARG
    assert b"selection" in lib.nasg_last_error()
    assert lib.nasg_create(ctypes.byref(_cfg(selection=1, mis_fraction=1.5)), ctypes.byref(st),
                           ctypes.byref(ctx)) == NASG_E_ARG
    assert b"mis_fraction" in lib.nasg_last_error()


def test_selection_sizes(lib):
    """8K + 1 outputs: 64 more weights; the BF16 packing adds one 16-row
    forward tile and 16 x 64 16x16x16 backward elements, FP32 one padded
    16-row block."""
    c = _cfg(selection=1)
    assert lib.nasg_num_weights(ctypes.byref(c)) == 21120 + 64
    assert lib.nasg_packed_bytes(ctypes.byref(c)) == 2 * (1024 + 3 * 4096 + 144 * 64 + 3 * 4096 + 8192 + 16 * 64)
    c32 = _cfg(precision=0, n_lobes=8, selection=1)
    assert lib.nasg_packed_bytes(ctypes.byref(c32)) == 4 * (64 * 17 + 3 * 64 * 65 + 80 * 65)


def test_encoded_network_sizes(lib):
    """The paper's default network (Sec. 4.1, Sec. 6): W_0 [128][64] on the
    encoded input, 8 lobes plus the selection output. BF16 packing: layer 0
    as 16x16x32 fragments (64 x 128), three hidden layers forward and
    backward, the output layer's 80 padded rows forward, its 64 lobe rows and
    the selection tile backward; the workspace holds 80 BF16 raw-output
    gradients per sample of a batch."""
    from oracle import mlp
    from paper_2303_08064_amd._lib import State, NASG_E_ARG
    c = _cfg(hidden=128, n_lobes=8, selection=1, encoding=1, max_batch=4096)
    nw = sum(o * i for (o, i) in mlp.layer_shapes(128, 4, 8, selection=True, encoded=True))
    assert nw == 65664 and lib.nasg_num_weights(ctypes.byref(c)) == nw
    H = 128
    assert lib.nasg_packed_bytes(ctypes.byref(c)) == 2 * (64 * H + 3 * H * H + 80 * H + 3 * H * H + 64 * H + 16 * H)
    assert lib.nasg_workspace_bytes(ctypes.byref(c)) >= 256 * nw * 4 + 4096 * 80 * 2
    # FP32: row-major layers with odd pitches (65 for layer 0, 129 after), 80 output rows
    c32 = _cfg(hidden=128, n_lobes=8, selection=1, encoding=1, precision=0, max_batch=4096)
    assert lib.nasg_packed_bytes(ctypes.byref(c32)) == 4 * (128 * 65 + 3 * 128 * 129 + 80 * 129)
    assert lib.nasg_workspace_bytes(ctypes.byref(c32)) >= 256 * nw * 4 + 4096 * 80 * 4
    # only that combination carries the encoded input
    for kw in (dict(hidden=64, n_lobes=8, selection=1, encoding=1),
               dict(hidden=128, n_lobes=8, selection=0, encoding=1),
               dict(hidden=128, n_lobes=32, selection=0, encoding=1),
               dict(hidden=128, n_lobes=8, selection=1, encoding=0),
               dict(hidden=128, n_lobes=8, selection=1, encoding=2)):
        assert lib.nasg_packed_bytes(ctypes.byref(_cfg(**kw))) == 0, kw
    ctx = ctypes.c_void_p()
    assert lib.nasg_create(ctypes.byref(_cfg(encoding=1)), ctypes.byref(State()), ctypes.byref(ctx)) == NASG_E_ARG
    assert b"encoded" in lib.nasg_last_error()


def test_blend_ramp_matches_oracle(lib):
    """nasg_blend_ramp (host) against the oracle's ramp of Sec. 5."""
    from oracle import train
    for n in (0, 1, 3, 4, 5, 63, 64, 100, 255, 256, 257, 10 ** 6):
        assert abs(lib.nasg_blend_ramp(n, 4, 64) - train.blend_ramp(n)) < 1e-7
    assert lib.nasg_blend_ramp(9, 3, 2) == train.blend_ramp(9, M=3, B=2) == 1.0
    assert lib.nasg_blend_ramp(-5, 4, 64) == 0.0 and lib.nasg_blend_ramp(10, 0, 64) == 0.0
