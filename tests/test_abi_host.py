"""The C ABI on the host: every declared symbol is exported, and argument
validation rejects bad calls before any HIP call (so these run without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_2202_02019_amd as P
from paper_2202_02019_amd import ladder as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ladder.h")

EINVAL, EWORKSPACE, EUNSUPPORTED = -1, -2, -3
FAKE = 1 << 20  # a 256-aligned non-NULL address that is never dereferenced on these paths


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ladder_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported():
    names = declared_functions()
    assert len(names) >= 10
    lib = ctypes.CDLL(P.library_path())
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(B.EXPORTS)


def _lib():
    return B._load()


def _opts(**kw):
    o = B.Options(**kw).c()
    return ctypes.byref(o)


def fwd(o=2, v=3, n=4, L=FAKE, tau=2 * FAKE, tbar=3 * FAKE, beta=0.0, R=4 * FAKE, E=None, ws=8 * FAKE, wsb=1 << 40,
        opts=None):
    return _lib().ladder_forward(o, v, n, L, tau, tbar, beta, R, E, ws, wsb, opts or _opts(), None)


def test_forward_validation():
    assert fwd(o=0) == EINVAL
    assert fwd(v=-1) == EINVAL
    assert fwd(n=0) == EINVAL
    assert fwd(o=1 << 21) == EINVAL
    assert fwd(L=None) == EINVAL
    assert fwd(tau=None) == EINVAL
    assert fwd(R=None) == EINVAL
    assert fwd(ws=None) == EINVAL
    assert fwd(tbar=None, E=5 * FAKE) == EINVAL                 # energy needs tbar
    assert fwd(L=FAKE + 4) == EINVAL                             # misaligned
    assert fwd(ws=8 * FAKE + 8) == EINVAL                        # ws needs 256-byte alignment
    assert fwd(wsb=16) == EWORKSPACE
    assert "workspace" in _lib().ladder_last_error().decode()
    assert fwd(R=2 * FAKE) == EINVAL                             # R aliases tau
    assert fwd(R=8 * FAKE) == EINVAL                             # R inside the workspace
    assert fwd(opts=_opts(precision=7)) == EUNSUPPORTED
    assert fwd(opts=_opts(flags=1 << 9)) == EUNSUPPORTED
    assert fwd(opts=_opts(n_abatch=-2)) == EINVAL
    assert "n_abatch" in _lib().ladder_last_error().decode()


def test_adjoint_validation():
    lib = _lib()
    ok = dict(o=2, v=3, n=4)

    def adj(L=FAKE, tau=2 * FAKE, w=3 * FAKE, X=4 * FAKE, ws=8 * FAKE, wsb=1 << 40, opts=None, **kw):
        d = dict(ok, **kw)
        return lib.ladder_adjoint(d["o"], d["v"], d["n"], L, tau, w, 1.0, 0.0, X, ws, wsb, opts or _opts(), None)

    assert adj(o=-3) == EINVAL
    assert adj(w=None) == EINVAL
    assert adj(X=FAKE) == EINVAL                                 # X aliases L
    assert adj(X=4 * FAKE + 2) == EINVAL
    assert adj(wsb=0) == EWORKSPACE
    assert adj(opts=_opts(precision=-1)) == EUNSUPPORTED


def test_tau_gradient_validation():
    lib = _lib()
    o, v, n = 2, 3, 4

    def tg(L=FAKE, w=2 * FAKE, G=4 * FAKE, ws=8 * FAKE, wsb=1 << 40, opts=None, **kw):
        d = dict(dict(o=o, v=v, n=n), **kw)
        return lib.ladder_tau_gradient(d["o"], d["v"], d["n"], L, w, 0.0, G, ws, wsb, opts or _opts(), None)

    assert tg(n=0) == EINVAL
    assert tg(L=None) == EINVAL
    assert tg(w=None) == EINVAL
    assert tg(G=None) == EINVAL
    assert tg(G=2 * FAKE) == EINVAL                              # G aliases w
    assert tg(G=FAKE + 16) == EINVAL                             # G overlaps L
    assert tg(ws=8 * FAKE + 64) == EINVAL
    assert tg(opts=_opts(precision=3)) == EUNSUPPORTED
    # the workspace holds the forward's plus the transposed L
    fb, tb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.ladder_workspace_size(o, v, n, _opts(), ctypes.byref(fb)) == 0
    assert lib.ladder_tau_gradient_workspace_size(o, v, n, _opts(), ctypes.byref(tb)) == 0
    assert tb.value >= v * v * n * 8
    assert tg(wsb=tb.value - 1) == EWORKSPACE
    assert lib.ladder_tau_gradient_workspace_size(o, v, n, _opts(), None) == EINVAL


def test_intermediate_entry_validation():
    lib = _lib()
    v, n = 3, 4
    assert lib.ladder_metric_contraction(0, n, FAKE, 2 * FAKE, 1.0, 0.0, 3 * FAKE, None) == EINVAL
    assert lib.ladder_metric_contraction(v, n, None, 2 * FAKE, 1.0, 0.0, 3 * FAKE, None) == EINVAL
    assert lib.ladder_metric_contraction(v, n, FAKE, 2 * FAKE, 1.0, 0.0, 2 * FAKE + 8, None) == EINVAL  # V overlaps W
    b = ctypes.c_size_t(0)
    assert lib.ladder_back_transform_workspace_size(v, n, ctypes.byref(b)) == 0 and b.value >= v * v * n * 8
    assert lib.ladder_back_transform_workspace_size(v, 0, ctypes.byref(b)) == EINVAL

    def bt(x=FAKE, y=2 * FAKE, W=3 * FAKE, Wmo=4 * FAKE, ws=8 * FAKE, wsb=1 << 30, vv=v):
        return lib.ladder_back_transform(vv, n, x, y, W, 1.0, 0.0, Wmo, ws, wsb, None)

    assert bt(vv=-1) == EINVAL
    assert bt(y=None) == EINVAL
    assert bt(Wmo=3 * FAKE) == EINVAL                            # Wmo aliases W
    assert bt(ws=8 * FAKE + 8) == EINVAL
    assert bt(wsb=8) == EWORKSPACE
    assert bt(ws=3 * FAKE) == EINVAL                             # workspace overlaps W


def test_ov3_abci_validation():
    """The OV^3 entry points reject bad dimensions, missing operands, overlaps, misalignment
    and a short workspace before any HIP call; the workspace holds the reordered multipliers,
    one [o][v][n] intermediate and the reordered Zvv."""
    lib = _lib()
    o, v, n = 2, 3, 4
    b = ctypes.c_size_t(0)
    assert lib.ladder_ov3_abci_workspace_size(o, v, n, ctypes.byref(b)) == 0
    assert b.value >= 8 * (o * o * v * v + o * v * n + v * v * n) and b.value % 256 == 0
    assert lib.ladder_ov3_abci_workspace_size(o, 0, n, ctypes.byref(b)) == EINVAL
    assert lib.ladder_ov3_abci_workspace_size(o, v, n, None) == EINVAL
    M = 1 << 24  # 16 MiB apart: no two arrays below overlap

    def call(L2=FAKE, R1=FAKE + M, Zvv=FAKE + 2 * M, Zvo=FAKE + 3 * M, Wab=FAKE + 4 * M, Wci=FAKE + 5 * M,
             ws=FAKE + 6 * M, wsb=1 << 20, oo=o):
        return lib.ladder_ov3_abci(oo, v, n, L2, R1, Zvv, Zvo, 1.0, 0.0, Wab, Wci, ws, wsb, None)

    assert call(oo=0) == EINVAL
    assert call(L2=None) == EINVAL
    assert call(R1=None) == EINVAL
    assert call(Wab=None, Wci=None) == EINVAL                   # nothing to compute
    assert call(Zvo=None) == EINVAL                             # Wab needs Zvo
    assert call(Zvv=None) == EINVAL                             # Wci needs Zvv
    assert call(Wab=FAKE + 8) == EINVAL                         # Wab overlaps L2
    assert call(Wci=FAKE + 4 * M + 8) == EINVAL                 # the outputs overlap
    assert call(ws=FAKE + 6 * M + 8) == EINVAL                  # misaligned workspace
    assert call(Wab=FAKE + 4 * M + 4) == EINVAL                 # misaligned output
    assert call(ws=FAKE + 3 * M) == EINVAL                      # workspace overlaps Zvo
    assert call(wsb=64) == EWORKSPACE
    assert lib.ladder_metric_contraction_pairs(0, n, FAKE, 2 * FAKE, 1.0, 0.0, 3 * FAKE, None) == EINVAL
    assert lib.ladder_metric_contraction_pairs(6, n, FAKE, None, 1.0, 0.0, 3 * FAKE, None) == EINVAL
    assert lib.ladder_metric_contraction_pairs(6, n, FAKE, 2 * FAKE, 1.0, 0.0, FAKE + 8, None) == EINVAL  # V overlaps Z


def test_ov3_abic_validation():
    """ladder_ov3_abic rejects bad calls before any HIP call."""
    lib = _lib()
    o, v, n = 2, 3, 4
    b = ctypes.c_size_t(0)
    assert lib.ladder_ov3_abic_workspace_size(o, v, n, None, ctypes.byref(b)) == 0
    assert b.value >= 8 * (3 * o * o * v * v + o ** 3 * v + v ** 3 + v * v * n) and b.value % 256 == 0
    bs = ctypes.c_size_t(0)
    assert lib.ladder_ov3_abic_workspace_size(o, v, n, _opts(precision=B.SPLIT_BF16), ctypes.byref(bs)) == 0
    assert bs.value > b.value                                   # plus the BF16 slices
    assert lib.ladder_ov3_abic_workspace_size(0, v, n, None, ctypes.byref(b)) == EINVAL
    assert lib.ladder_ov3_abic_workspace_size(o, v, n, _opts(precision=7), ctypes.byref(b)) == EUNSUPPORTED
    M = 1 << 24

    def call(L1=FAKE, L2=FAKE + M, T=FAKE + 2 * M, R1=FAKE + 3 * M, R2=FAKE + 4 * M, Zvv=FAKE + 5 * M,
             Zov=FAKE + 6 * M, Wab=FAKE + 7 * M, Wic=FAKE + 8 * M, ws=FAKE + 9 * M, wsb=1 << 22, vv=v, opts=None):
        return lib.ladder_ov3_abic(o, vv, n, 0.5, L1, L2, T, R1, R2, Zvv, Zov, 1.0, 0.0, Wab, Wic, ws, wsb, opts, None)

    assert call(vv=0) == EINVAL
    for k in ("L1", "L2", "T", "R1", "R2", "ws"):
        assert call(**{k: None}) == EINVAL, k
    assert call(Wab=None, Wic=None) == EINVAL
    assert call(Zov=None) == EINVAL                             # Wab needs Zov
    assert call(Zvv=None) == EINVAL                             # Wic needs Zvv
    assert call(T=FAKE + 2 * M + 4) == EINVAL                   # misaligned input
    assert call(ws=FAKE + 9 * M + 64) == EINVAL                 # misaligned workspace
    assert call(Wab=FAKE + 4 * M + 8) == EINVAL                 # Wab overlaps R2
    assert call(Wic=FAKE + 7 * M + 8) == EINVAL                 # the outputs overlap
    assert call(ws=FAKE + 2 * M) == EINVAL                      # workspace overlaps T
    assert call(wsb=256) == EWORKSPACE
    assert call(wsb=b.value, opts=_opts(precision=B.SPLIT_BF16)) == EWORKSPACE   # FP64 size is short for split
    assert call(opts=_opts(precision=B.SPLIT_BF16, n_slices=9)) == EUNSUPPORTED


def test_mfma_probe_validation():
    lib = _lib()
    fl = ctypes.c_double(0.0)
    assert lib.ladder_mfma_probe(7, 10, 4, FAKE, ctypes.byref(fl), None) == EUNSUPPORTED
    assert lib.ladder_mfma_probe(B.PROBE_BF16, 0, 4, FAKE, ctypes.byref(fl), None) == EINVAL
    assert lib.ladder_mfma_probe(B.PROBE_FP64, 10, 0, FAKE, ctypes.byref(fl), None) == EINVAL
    assert lib.ladder_mfma_probe(B.PROBE_FP64, 10, 4, None, ctypes.byref(fl), None) == EINVAL
    assert lib.ladder_mfma_probe(B.PROBE_FP64, 10, 4, FAKE + 4, ctypes.byref(fl), None) == EINVAL


def test_autotune_validation_and_cache(tmp_path):
    """Argument checks run before any HIP call; the cache file is parsed line by line (other
    devices' lines and junk are skipped) and a tuned batch size changes the ragged-batch plan."""
    import torch
    lib = _lib()
    nA = ctypes.c_int64(0)

    def tune(opts=None, tbar=3 * FAKE, X=5 * FAKE, wsb=1 << 40):
        return lib.ladder_autotune(4, 20, 60, FAKE, 2 * FAKE, tbar, 4 * FAKE, X, 8 * FAKE, wsb, opts or _opts(),
                                   None, ctypes.byref(nA), None)

    assert tune(opts=_opts(n_abatch=3)) == EINVAL
    assert tune(tbar=None) == EINVAL
    assert tune(X=FAKE) == EINVAL                                # X aliases L
    assert tune(wsb=64) == EWORKSPACE
    assert lib.ladder_autotune_load(None, None) == EINVAL
    assert lib.ladder_autotune_load(str(tmp_path / "missing.jsonl").encode(), None) == EINVAL
    if torch.cuda.is_available():
        pytest.skip("the cache lines below are written for a host without a GPU (device tag 'unknown')")
    f = tmp_path / "tune.jsonl"
    f.write_text('{"device": "unknown", "o": 4, "v": 20, "n": 60, "precision": 0, "n_slices": 0, "flags": 0, '
                 '"n_abatch": 3, "est_ms": 1.0}\n'
                 '{"device": "gfx950:256", "o": 4, "v": 20, "n": 60, "precision": 0, "n_slices": 0, "flags": 0, '
                 '"n_abatch": 7, "est_ms": 1.0}\n'
                 'not a cache line\n'
                 '{"device": "unknown", "o": 4, "v": 20, "n": 60, "precision": 0, "n_slices": 0, "flags": 0, '
                 '"n_abatch": 999, "est_ms": 1.0}\n')
    arr = (B._CInstance * 1)()
    arr[0] = B._CInstance(4, 20, 60, FAKE, 2 * FAKE, 3 * FAKE, 4 * FAKE, 5 * FAKE, 6 * FAKE)

    def bws():
        b = ctypes.c_size_t(0)
        assert lib.ladder_batched_workspace_size(1, arr, 3, _opts(), ctypes.byref(b)) == 0
        return b.value

    P.autotune_reset()
    before = bws()
    assert P.autotune_load(str(f)) == 1                          # the foreign device, junk and n_abatch > v are skipped
    tuned = bws()
    P.autotune_reset()
    assert bws() == before
    assert tuned < before                                        # 3 virtual indices per batch instead of 10


def test_amplitude_entry_validation():
    lib = _lib()
    assert lib.ladder_mp2_amplitudes(0, 2, 2, FAKE, 2 * FAKE, 3 * FAKE, None) == EINVAL
    assert lib.ladder_mp2_amplitudes(2, 2, 2, FAKE, 2 * FAKE, None, None) == EINVAL
    assert lib.ladder_mp2_amplitudes(2, 2, 2, FAKE, 2 * FAKE, FAKE, None) == EINVAL  # t overlaps Lov
    assert lib.ladder_amplitude_update(2, 2, None, FAKE, 2 * FAKE, None) == EINVAL
    assert lib.ladder_amplitude_update(2, 2, 3 * FAKE, FAKE + 8, FAKE, None) == EINVAL  # partial overlap
    assert lib.ladder_excited_amplitudes(2, 2, 1.0, FAKE, 2 * FAKE, 2, 3 * FAKE, None) == EUNSUPPORTED  # mode
    assert lib.ladder_excited_amplitudes(2, 2, 1.0, None, 2 * FAKE, 0, 3 * FAKE, None) == EINVAL
    assert lib.ladder_excited_amplitudes(2, 2, 1.0, FAKE, 2 * FAKE, 0, 2 * FAKE, None) == EINVAL  # U is R2
    assert lib.ladder_excited_amplitudes(2, 2, 1.0, FAKE, 2 * FAKE, 0, FAKE + 8, None) == EINVAL  # partial overlap


def test_strerror_and_options():
    lib = _lib()
    for code in (0, -1, -2, -3, -4, -99):
        assert lib.ladder_strerror(code)
    o = B._COptions()
    o.precision = 9
    lib.ladder_default_options(ctypes.byref(o))
    assert o.precision == 0 and o.n_abatch == 0 and o.flags == 0
    with pytest.raises(P.LadderError):
        P.workspace_size(0, 1, 1)


@pytest.mark.parametrize("o,v,n", [(78, 657, 2200), (40, 350, 1200), (20, 150, 600), (4, 20, 60)])
def test_workspace_never_holds_full_v4(o, v, n):
    """The V^4 arrays g and D are only ever held as batch tiles (Sec. II B, Appendix A storage policy)."""
    ws = P.workspace_size(o, v, n)
    if v > 20:
        assert ws < 8 * v ** 4
    # one virtual index per batch: the g/D tile and its packed halves (v^3 each) plus
    # packed copies of the amplitudes (o^2 v^2); nothing of size v^4
    for flags in (0, P.FLAG_DENSE):
        ws1 = P.workspace_size(o, v, n, P.Options(n_abatch=1, flags=flags))
        assert ws1 < 16 * v ** 3 + 16 * o * o * v * v + (1 << 24)


def test_batched_validation():
    lib = _lib()
    arr = (B._CInstance * 2)()
    arr[0] = B._CInstance(2, 3, 4, FAKE, 2 * FAKE, 3 * FAKE, 4 * FAKE, 0, 6 * FAKE)
    arr[1] = B._CInstance(2, 0, 4, FAKE, 2 * FAKE, 3 * FAKE, 4 * FAKE, 0, 6 * FAKE)
    sz = ctypes.c_size_t(0)
    assert lib.ladder_batched_workspace_size(0, arr, 3, _opts(), ctypes.byref(sz)) == EINVAL
    assert lib.ladder_batched_workspace_size(1, arr, 0, _opts(), ctypes.byref(sz)) == EINVAL
    assert lib.ladder_batched_workspace_size(2, arr, 3, _opts(), ctypes.byref(sz)) == EINVAL  # v = 0
    assert "instance 1" in lib.ladder_last_error().decode()
    assert lib.ladder_batched_workspace_size(1, arr, 3, _opts(), ctypes.byref(sz)) == 0 and sz.value > 0
    arr[0].R = None
    assert lib.ladder_batched_workspace_size(1, arr, 1, _opts(), ctypes.byref(sz)) == EINVAL
    assert lib.ladder_batched(1, arr, 2, 8 * FAKE, 16, _opts(), None) == EWORKSPACE


def test_gemm_validation():
    lib = _lib()
    SPLIT = 1

    def gm(M=3, N=4, K=5, A=FAKE, lda=5, B=2 * FAKE, ldb=5, C=4 * FAKE, ldc=4, ws=8 * FAKE, wsb=1 << 40, opts=None):
        return lib.ladder_gemm(M, N, K, 1.0, A, lda, B, ldb, 0.0, C, ldc, ws, wsb, opts or _opts(), None)

    assert gm(M=0) == EINVAL
    assert gm(K=-1) == EINVAL
    assert gm(N=(1 << 31) + 1) == EINVAL
    assert gm(A=None) == EINVAL
    assert gm(C=None) == EINVAL
    assert gm(lda=4) == EINVAL                                   # lda < K
    assert gm(ldc=3) == EINVAL                                   # ldc < N
    assert gm(B=2 * FAKE + 4) == EINVAL                          # misaligned
    assert gm(C=FAKE) == EINVAL                                  # C aliases A
    assert gm(opts=_opts(precision=7)) == EUNSUPPORTED
    assert gm(opts=_opts(precision=SPLIT, n_slices=9)) == EUNSUPPORTED
    assert gm(ws=None, opts=_opts(precision=SPLIT)) == EINVAL      # split needs a workspace
    assert gm(ws=8 * FAKE + 64, opts=_opts(precision=SPLIT)) == EINVAL
    assert gm(wsb=64, opts=_opts(precision=SPLIT)) == EWORKSPACE
    assert gm(C=8 * FAKE, opts=_opts(precision=SPLIT)) == EINVAL   # C inside the workspace
    b = ctypes.c_size_t(7)
    assert lib.ladder_gemm_workspace_size(3, 4, 5, _opts(), ctypes.byref(b)) == 0 and b.value == 0
    assert lib.ladder_gemm_workspace_size(3, 4, 5, _opts(precision=SPLIT, n_slices=3), ctypes.byref(b)) == 0
    # slices of two one-panel operands (3 slices x 128 rows x 16 k x 2 bytes) plus one exponent chunk each
    assert b.value == 2 * (3 * 128 * 16 * 2 + 256)
    assert lib.ladder_gemm_workspace_size(3, 4, 0, _opts(), ctypes.byref(b)) == EINVAL


def test_forward_noalloc_validation():
    """Sizes beyond the static scratch are refused on the host, before any HIP call."""
    lib = _lib()
    S = ctypes.c_void_p

    def nf(o=2, v=3, n=4, L=FAKE, tau=2 * FAKE, tbar=3 * FAKE, R=4 * FAKE, E=None, opts=None):
        return lib.ladder_forward_noalloc(o, v, n, S(L), S(tau), S(tbar), 0.0, S(R), S(E), opts or _opts(), None)

    assert nf(o=0) == EINVAL
    assert nf(opts=_opts(precision=7)) == EUNSUPPORTED
    # the packed amplitudes alone (o^2 v^2 / 2 doubles, about 1.3 GB here) exceed 256 MiB
    assert nf(o=100, v=400, n=10) == EWORKSPACE
    assert "static scratch" in lib.ladder_last_error().decode()
    # an explicit batch whose tile does not fit is refused, not shrunk
    assert nf(o=2, v=200, n=8, opts=_opts(n_abatch=200, flags=2)) == EWORKSPACE
    assert nf(L=None) == EINVAL
    assert nf(R=2 * FAKE) == EINVAL                             # R aliases tau
    assert nf(tbar=None, E=5 * FAKE) == EINVAL                  # energy needs tbar


def test_adjoint_slice_count_option():
    """n_slices_adjoint: 0 means n_slices; 2..6 otherwise (split only); it sizes the adjoint region."""
    SPLIT = 1
    assert fwd(opts=_opts(precision=SPLIT, n_slices_adjoint=7)) == EUNSUPPORTED
    assert fwd(opts=_opts(precision=SPLIT, n_slices_adjoint=1)) == EUNSUPPORTED
    assert fwd(opts=_opts(n_slices_adjoint=-1)) == EINVAL
    o, v, n = 6, 40, 90
    w44 = P.workspace_size(o, v, n, P.Options(precision=SPLIT, n_slices=4, n_abatch=4))
    w45 = P.workspace_size(o, v, n, P.Options(precision=SPLIT, n_slices=4, n_slices_adjoint=5, n_abatch=4))
    w55 = P.workspace_size(o, v, n, P.Options(precision=SPLIT, n_slices=5, n_abatch=4))
    w54 = P.workspace_size(o, v, n, P.Options(precision=SPLIT, n_slices=5, n_slices_adjoint=4, n_abatch=4))
    assert w44 < w45 <= w55 and w44 < w54 <= w55
    # in FP64 the field is ignored
    assert P.workspace_size(o, v, n, P.Options(n_slices_adjoint=3)) == P.workspace_size(o, v, n)


def test_int8_precision_option():
    """LADDER_SPLIT_INT8: the same slice-count rules as BF16; its slices take one byte per
    element and 32-k blocks, so a one-panel ladder_gemm operand is 128 rows x 32 k bytes per
    slice, and the forward's workspace is below the BF16 one at the same counts."""
    INT8 = 2
    assert P.SPLIT_INT8 == INT8 and P.PROBE_INT8 == 2
    assert fwd(opts=_opts(precision=INT8, n_slices=7)) == EUNSUPPORTED
    assert fwd(opts=_opts(precision=INT8, n_slices=1)) == EUNSUPPORTED
    assert fwd(opts=_opts(precision=INT8, n_slices_adjoint=7)) == EUNSUPPORTED
    assert fwd(opts=_opts(precision=3)) == EUNSUPPORTED
    lib = _lib()
    b = ctypes.c_size_t(0)
    assert lib.ladder_gemm_workspace_size(3, 4, 5, _opts(precision=INT8, n_slices=3), ctypes.byref(b)) == 0
    assert b.value == 2 * (3 * 128 * 32 + 256)
    o, v, n = 6, 40, 90
    w8 = P.workspace_size(o, v, n, P.Options(precision=INT8, n_slices=5, n_slices_adjoint=5, n_abatch=4,
                                             flags=P.FLAG_DENSE))
    w16 = P.workspace_size(o, v, n, P.Options(precision=1, n_slices=5, n_slices_adjoint=5, n_abatch=4,
                                              flags=P.FLAG_DENSE))
    assert w8 < w16
    fl = ctypes.c_double(0.0)
    assert lib.ladder_mfma_probe(INT8, 0, 4, FAKE, ctypes.byref(fl), None) == EINVAL
