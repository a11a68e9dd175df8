"""GPU-side draws of the synthetic recipe (libsynth.so), same definition as generate.py."""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import torch

from .generate import L_SCALE, NOISE_SCALE

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libsynth.so")
_lib = None


def build() -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", tmp, os.path.join(HERE, "synth.hip")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed for synth.hip:\n" + res.stderr)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError("libsynth.so is not built; run synthetic.gpu.build()")
        lib = ctypes.CDLL(LIB)
        u64, i64, dbl, vp = ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        lib.synth_L_block.argtypes = [u64, i64, i64, i64, i64, i64, i64, dbl, vp, vp]
        lib.synth_eps.argtypes = [u64, i64, i64, vp, vp]
        lib.synth_add_noise.argtypes = [u64, i64, i64, dbl, vp, vp, vp]
        for f in ("synth_L_block", "synth_eps", "synth_add_noise"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _st():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ok(rc, what):
    if rc != 0:
        raise RuntimeError("%s failed (%d)" % (what, rc))


def draw_L_vv(seed, o, v, n, device="cuda"):
    out = torch.empty((v, v, n), dtype=torch.float64, device=device)
    _ok(_load().synth_L_block(seed, o + v, n, o, v, o, v, L_SCALE / math.sqrt(n), ctypes.c_void_p(out.data_ptr()),
                              _st()), "synth_L_block")
    return out


def draw_L_ov(seed, o, v, n, device="cuda"):
    out = torch.empty((o, v, n), dtype=torch.float64, device=device)
    _ok(_load().synth_L_block(seed, o + v, n, 0, o, o, v, L_SCALE / math.sqrt(n), ctypes.c_void_p(out.data_ptr()),
                              _st()), "synth_L_block")
    return out


def draw_eps(seed, o, v, device="cuda"):
    out = torch.empty((o + v,), dtype=torch.float64, device=device)
    _ok(_load().synth_eps(seed, o, v, ctypes.c_void_p(out.data_ptr()), _st()), "synth_eps")
    return out


def add_noise(seed, o, v, t, out=None):
    """out = t + 1e-2 * xi (pair-symmetric noise)."""
    if out is None:
        out = torch.empty_like(t)
    _ok(_load().synth_add_noise(seed, o, v, NOISE_SCALE, ctypes.c_void_p(t.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()), _st()), "synth_add_noise")
    return out
