"""The C ABI without a GPU: the library loads, exports every function nnls.h declares, sizes
workspaces, and rejects bad arguments on the host before any HIP call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nnls.h")
LIB = os.path.join(ROOT, "paper_1502_01645_amd", "libnnls.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(nnls_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        from paper_1502_01645_amd import build
        build.build()
    from paper_1502_01645_amd import nnls
    return nnls.lib()


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ["nnls_prepare", "nnls_solve", "nnls_refine", "nnls_workspace_bytes"]:
        assert required in names


def test_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_workspace_sizes(L, monkeypatch):
    from paper_1502_01645_amd import nnls as N
    # FP32 with several right-hand sides: matrix-core solver, only a queue counter
    assert N.workspace_bytes(N.OP_SOLVE, 0, 100, 3, 0, N.F32) >= 4
    # FP64, or the per-column solver forced: three vectors per column
    assert N.workspace_bytes(N.OP_SOLVE, 0, 100, 3, 0, N.F64) >= 3 * 100 * 3 * 8
    monkeypatch.setenv("NNLS_SOLVER", "wg")
    assert N.workspace_bytes(N.OP_SOLVE, 0, 100, 3, 0, N.F32) >= 3 * 100 * 3 * 4
    monkeypatch.delenv("NNLS_SOLVER")
    assert N.workspace_bytes(N.OP_SCALES, 1000, 100, 0, 0, N.F32) > 0
    assert N.workspace_bytes(N.OP_PREPARE, 1000, 100, 1, N.GRAM_BF16X3, N.F32) > 0
    assert N.workspace_bytes(N.OP_REFINE, 1000, 100, 1, 0, N.F32) > 0
    # invalid shapes size to 0
    assert N.workspace_bytes(N.OP_SOLVE, 0, 0, 3, 0, N.F32) == 0
    assert N.workspace_bytes(N.OP_SOLVE, 0, 10, 3, 0, 7) == 0
    assert N.workspace_bytes(99, 10, 10, 3, 0, N.F32) == 0


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first


def test_prepare_rejects_bad_arguments(L):
    from paper_1502_01645_amd import nnls as N
    ws = ctypes.c_size_t(1 << 40)
    cases = [
        dict(d=0), dict(n=0), dict(k=-1), dict(lda=5), dict(ldb=0), dict(A=None), dict(Q=None),
        dict(s=None), dict(B=None), dict(q=None), dict(dtype=5), dict(mode=N.GRAM_FP64),
        dict(mode=7),
    ]
    for c in cases:
        a = dict(d=100, n=10, k=2, A=FAKE, lda=10, B=FAKE, ldb=2, mode=N.GRAM_BF16X3, dtype=N.F32,
                 Q=FAKE, q=FAKE, s=FAKE)
        a.update(c)
        rc = L.nnls_prepare(a["d"], a["n"], a["k"], a["A"], a["lda"], a["B"], a["ldb"], a["mode"],
                            a["dtype"], a["Q"], a["q"], a["s"], FAKE, ws, None)
        assert rc == N.E_ARG, c
    # FP64 data must use the FP64 Gram
    rc = L.nnls_prepare(100, 10, 2, FAKE, 10, FAKE, 2, N.GRAM_BF16X3, N.F64, FAKE, FAKE, FAKE, FAKE,
                        ws, None)
    assert rc == N.E_ARG
    # workspace too small
    rc = L.nnls_prepare(100, 10, 2, FAKE, 10, FAKE, 2, N.GRAM_BF16X3, N.F32, FAKE, FAKE, FAKE, FAKE,
                        0, None)
    assert rc == N.E_WORKSPACE


def test_solve_rejects_bad_arguments(L):
    from paper_1502_01645_amd import nnls as N
    big = 1 << 40
    base = dict(n=10, k=2, dt=N.F32, Q=FAKE, q=FAKE, tol=1e-5, mi=0, X=FAKE, it=FAKE, kkt=FAKE,
                st=FAKE, tr=None, tl=0, ws=FAKE, wsb=big)
    cases = [dict(n=0), dict(k=0), dict(dt=3), dict(Q=None), dict(q=None), dict(X=None),
             dict(it=None), dict(kkt=None), dict(st=None), dict(tol=-1.0), dict(tol=float("nan")),
             dict(tol=float("inf")), dict(mi=-1), dict(tl=-1), dict(tr=FAKE, tl=0)]
    for c in cases:
        a = dict(base)
        a.update(c)
        rc = L.nnls_solve(a["n"], a["k"], a["dt"], a["Q"], a["q"], None, a["tol"], a["mi"], None,
                          a["X"], a["it"], a["kkt"], a["st"], None, a["tr"], a["tl"], a["ws"],
                          a["wsb"], None)
        assert rc == N.E_ARG, c
    rc = L.nnls_solve(10, 2, N.F32, FAKE, FAKE, None, 1e-5, 0, None, FAKE, FAKE, FAKE, FAKE, None,
                      None, 0, FAKE, 4, None)
    assert rc == N.E_WORKSPACE
    rc = L.nnls_solve(10, 2, N.F32, FAKE, FAKE, None, 1e-5, 0, None, FAKE, FAKE, FAKE, FAKE, None,
                      None, 0, None, big, None)
    assert rc == N.E_WORKSPACE
    # a trace with a length passes the checks (and a NULL trace ignores its length)
    for tr, tl in [(FAKE, 5), (None, 7)]:
        rc = L.nnls_solve(10, 2, N.F32, FAKE, FAKE, None, 1e-5, 0, None, FAKE, FAKE, FAKE, FAKE,
                          None, tr, tl, FAKE, 4, None)
        assert rc == N.E_WORKSPACE


def test_split_prepare_rejects_bad_arguments(L):
    from paper_1502_01645_amd import nnls as N
    big = 1 << 40
    assert L.nnls_column_scales(0, 10, FAKE, 10, N.F32, FAKE, FAKE, big, None) == N.E_ARG
    assert L.nnls_column_scales(10, 10, None, 10, N.F32, FAKE, FAKE, big, None) == N.E_ARG
    assert L.nnls_column_scales(10, 10, FAKE, 9, N.F32, FAKE, FAKE, big, None) == N.E_ARG
    assert L.nnls_column_scales(10, 10, FAKE, 10, N.F32, None, FAKE, big, None) == N.E_ARG
    assert L.nnls_column_scales(10, 10, FAKE, 10, N.F32, FAKE, FAKE, 0, None) == N.E_WORKSPACE
    assert L.nnls_gram_rescaled(10, 10, 1, FAKE, 10, FAKE, 1, N.GRAM_BF16X3, N.F32, None, FAKE,
                                FAKE, FAKE, big, None) == N.E_ARG
    assert L.nnls_gram_rescaled(10, 10, 1, FAKE, 10, None, 1, N.GRAM_BF16X3, N.F32, FAKE, FAKE,
                                FAKE, FAKE, big, None) == N.E_ARG
    assert L.nnls_gram_rescaled(10, 10, 1, FAKE, 10, FAKE, 1, N.GRAM_FP64, N.F32, FAKE, FAKE,
                                FAKE, FAKE, big, None) == N.E_ARG
    # the unscaled Gram: same checks, no s
    assert L.nnls_gram(10, 10, 1, None, 10, FAKE, 1, N.GRAM_BF16X3, N.F32, FAKE, FAKE, FAKE, big,
                       None) == N.E_ARG
    assert L.nnls_gram(10, 10, 1, FAKE, 10, None, 1, N.GRAM_BF16X3, N.F32, FAKE, FAKE, FAKE, big,
                       None) == N.E_ARG
    assert L.nnls_gram(10, 10, 1, FAKE, 10, FAKE, 1, N.GRAM_BF16X3, N.F32, None, FAKE, FAKE, big,
                       None) == N.E_ARG
    assert L.nnls_gram(10, 10, 1, FAKE, 10, FAKE, 1, N.GRAM_FP64, N.F32, FAKE, FAKE, FAKE, big,
                       None) == N.E_ARG
    assert L.nnls_gram(10, 10, 1, FAKE, 10, FAKE, 1, N.GRAM_BF16X3, N.F32, FAKE, FAKE, FAKE, 0,
                       None) == N.E_WORKSPACE


def test_nmf_helpers_reject_bad_arguments(L):
    from paper_1502_01645_amd import nnls as N
    assert L.nnls_transpose(0, 5, FAKE, 5, FAKE, 1, None) == N.E_ARG
    assert L.nnls_transpose(5, 5, None, 5, FAKE, 5, None) == N.E_ARG
    assert L.nnls_transpose(5, 6, FAKE, 5, FAKE, 5, None) == N.E_ARG    # ld_src < cols
    assert L.nnls_transpose(5, 6, FAKE, 6, FAKE, 4, None) == N.E_ARG    # ld_dst < rows
    assert L.nnls_transpose(64 * 65536, 1, FAKE, 1, FAKE, 64 * 65536, None) == N.E_UNSUPPORTED
    assert L.nnls_rescale_start(0, 3, FAKE, FAKE, FAKE, None) == N.E_ARG
    assert L.nnls_rescale_start(3, 3, None, FAKE, FAKE, None) == N.E_ARG
    assert L.nnls_rescale_start(3, 3, FAKE, FAKE, None, None) == N.E_ARG


def test_solve_noalloc_rejects_bad_arguments_and_oversized_scratch(L):
    from paper_1502_01645_amd import nnls as N
    args = lambda n, k, dt, Q=FAKE, tol=1e-5: (n, k, dt, Q, FAKE, None, tol, 0, None, FAKE, FAKE,  # noqa
                                               FAKE, FAKE, None, None, 0, None)
    assert L.nnls_solve_noalloc(*args(0, 3, N.F32)) == N.E_ARG
    assert L.nnls_solve_noalloc(*args(10, 3, N.F32, Q=None)) == N.E_ARG
    assert L.nnls_solve_noalloc(*args(10, 3, N.F32, tol=-1.0)) == N.E_ARG
    assert L.nnls_solve_noalloc(*args(10, 3, 9)) == N.E_ARG
    # the per-column solver needs 12 n k (FP32) or 24 n k (FP64) bytes: past the fixed scratch
    # the call is refused before any device work
    assert L.nnls_solve_noalloc(*args(1001, 1000, N.F32)) == N.E_WORKSPACE
    assert L.nnls_solve_noalloc(*args(500, 1000, N.F64)) == N.E_WORKSPACE
    assert N.workspace_bytes(N.OP_SOLVE, 0, 500, 1000, 0, N.F64) > N.NOALLOC_SCRATCH_BYTES


def test_refine_rejects_bad_arguments(L):
    from paper_1502_01645_amd import nnls as N
    big = 1 << 40
    base = dict(d=50, n=10, k=2, A=FAKE, lda=10, B=FAKE, ldb=2, dt=N.F32, X=FAKE, kk=FAKE, ob=FAKE)
    for c in [dict(d=0), dict(n=0), dict(k=0), dict(A=None), dict(B=None), dict(X=None),
              dict(kk=None), dict(lda=9), dict(ldb=1), dict(dt=9)]:
        a = dict(base)
        a.update(c)
        rc = L.nnls_refine(a["d"], a["n"], a["k"], a["A"], a["lda"], a["B"], a["ldb"], a["dt"],
                           a["X"], a["kk"], a["ob"], FAKE, big, None)
        assert rc == N.E_ARG, c
    rc = L.nnls_refine(50, 10, 2, FAKE, 10, FAKE, 2, N.F32, FAKE, FAKE, FAKE, FAKE, 8, None)
    assert rc == N.E_WORKSPACE
    # obj64 may be NULL (the objective is then not formed): argument checks pass
    rc = L.nnls_refine(50, 10, 2, FAKE, 10, FAKE, 2, N.F32, FAKE, FAKE, None, FAKE, 8, None)
    assert rc == N.E_WORKSPACE


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1502_01645_amd import nnls as N
    monkeypatch.setattr(N, "_lib", None)
    monkeypatch.setattr(N, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(N.NNLSError):
        N.lib()


def test_batched_plan_rejects_bad_arguments(L):
    from paper_1502_01645_amd import nnls as N
    descs = (N.ProblemDesc * 2)(N.ProblemDesc(30, 10, 0, 0, 0, 0, 0),
                                N.ProblemDesc(30, 10, 300, 30, 100, 10, 10))
    assert L.nnls_batched_workspace_bytes(descs, 2) > 0
    assert L.nnls_batched_workspace_bytes(None, 2) == 0
    pools = [FAKE] * 6 + [FAKE, FAKE, FAKE, None]  # A B Q q s X pools, iters kkt status rows
    big = 1 << 40

    def create(d=descs, count=2, tol=1e-5, mi=0, p=pools, ws=FAKE, wsb=big, stream=FAKE):
        out = ctypes.c_void_p()
        return L.nnls_batched_plan_create(d, count, tol, mi, None, *p, ws, wsb, stream,
                                          ctypes.byref(out))

    assert create(count=0) == N.E_ARG
    assert create(d=None) == N.E_ARG
    assert create(tol=-1.0) == N.E_ARG
    assert create(mi=-3) == N.E_ARG
    assert create(stream=None) == N.E_ARG          # the null stream cannot be captured
    for j in range(9):
        p = list(pools)
        p[j] = None
        assert create(p=p) == N.E_ARG, j
    bad = (N.ProblemDesc * 1)(N.ProblemDesc(0, 10, 0, 0, 0, 0, 0))
    assert create(d=bad, count=1) == N.E_ARG
    big_n = (N.ProblemDesc * 1)(N.ProblemDesc(3000, 2000, 0, 0, 0, 0, 0))
    assert create(d=big_n, count=1) == N.E_UNSUPPORTED
    assert create(ws=None) == N.E_WORKSPACE
    assert create(wsb=16) == N.E_WORKSPACE


def test_autotune_rejects_bad_arguments(L):
    from paper_1502_01645_amd import nnls as N
    shapes = (ctypes.c_int64 * 4)(300, 100, 900, 300)
    assert L.nnls_autotune(None, N.TUNE_BATCHED, shapes, 2, None) == N.E_ARG
    assert L.nnls_autotune(b"/tmp/x.json", 7, shapes, 2, None) == N.E_ARG
    assert L.nnls_autotune(b"/tmp/x.json", N.TUNE_BATCHED, None, 2, None) == N.E_ARG
    assert L.nnls_autotune(b"/tmp/x.json", N.TUNE_BATCHED, shapes, 0, None) == N.E_ARG
    bad = (ctypes.c_int64 * 2)(300, 0)
    assert L.nnls_autotune(b"/tmp/x.json", N.TUNE_BATCHED, bad, 1, None) == N.E_ARG
    big = (ctypes.c_int64 * 2)(3000, 2000)
    assert L.nnls_autotune(b"/tmp/x.json", N.TUNE_BATCHED, big, 1, None) == N.E_UNSUPPORTED


def test_mlp_sizes_and_argument_errors(L):
    from paper_1502_01645_amd import nnls as N
    P = 256 * 1024 + 1024 + 1024 * 1024 + 1024 + 1024 * 256 + 256
    assert L.nnls_mlp_param_count() == P
    assert L.nnls_mlp_blob_bytes() == 14 * P + 8 * 256
    assert L.nnls_mlp_workspace_bytes(0, 0) == 0
    assert L.nnls_mlp_workspace_bytes(64, 1) > L.nnls_mlp_workspace_bytes(64, 0) > 0
    big = 1 << 40
    # batch not a multiple of 64, null pointers, workspace too small
    assert L.nnls_mlp_forward(65, FAKE, FAKE, FAKE, FAKE, big, None) == N.E_ARG
    assert L.nnls_mlp_forward(0, FAKE, FAKE, FAKE, FAKE, big, None) == N.E_ARG
    assert L.nnls_mlp_forward(64, None, FAKE, FAKE, FAKE, big, None) == N.E_ARG
    assert L.nnls_mlp_forward(64, FAKE, FAKE, FAKE, FAKE, 16, None) == N.E_WORKSPACE
    assert L.nnls_mlp_gradients(64, FAKE, FAKE, None, 0.01, None, None, FAKE, big,
                                None) == N.E_ARG
    assert L.nnls_mlp_gradients(64, FAKE, FAKE, FAKE, 0.01, None, None, FAKE, 16,
                                None) == N.E_WORKSPACE
    # Adam steps count from 1; the learning rate must be positive
    assert L.nnls_mlp_train_step(64, FAKE, FAKE, FAKE, 1e-3, 0, 0.01, None, FAKE, big,
                                 None) == N.E_ARG
    assert L.nnls_mlp_train_step(64, FAKE, FAKE, FAKE, 0.0, 1, 0.01, None, FAKE, big,
                                 None) == N.E_ARG
    assert L.nnls_mlp_reset_state(None, None) == N.E_ARG
    assert L.nnls_mlp_fit_input_workspace_bytes() > 0
    assert L.nnls_mlp_fit_input(0, FAKE, FAKE, FAKE, big, None) == N.E_ARG
    assert L.nnls_mlp_fit_input(10, FAKE, FAKE, FAKE, 8, None) == N.E_WORKSPACE
    # warm start: only n = 256
    assert L.nnls_warm_start_workspace_bytes(128, 4) == 0
    assert L.nnls_warm_start_workspace_bytes(256, 4) > 0
    assert L.nnls_warm_start(128, 4, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, big,
                             None) == N.E_UNSUPPORTED
    assert L.nnls_warm_start(0, 4, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, big, None) == N.E_ARG
    assert L.nnls_warm_start(256, 0, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, big, None) == N.E_ARG
    assert L.nnls_warm_start(256, 4, FAKE, FAKE, FAKE, FAKE, None, FAKE, big, None) == N.E_ARG
    assert L.nnls_warm_start(256, 4, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, 16,
                             None) == N.E_WORKSPACE
    assert L.nnls_mlp_inputs(128, 4, FAKE, None, FAKE, None, None) == N.E_UNSUPPORTED
    assert L.nnls_mlp_inputs(256, 4, FAKE, FAKE, FAKE, None, None) == N.E_ARG
    assert L.nnls_mlp_inputs(256, 0, FAKE, None, FAKE, None, None) == N.E_ARG


_PAYLOAD = {}


def _checkpoint_bytes(L, **over):
    """A checkpoint file as nnls.h describes it, with a valid FNV-1a hash of its payload (header
    fields overridable)."""
    import struct
    nbytes = int(L.nnls_mlp_blob_bytes())
    if nbytes not in _PAYLOAD:
        payload = bytes(range(256)) * (nbytes // 256) + bytes(nbytes % 256)
        h = 0xcbf29ce484222325
        for c in payload:
            h = ((h ^ c) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
        _PAYLOAD[nbytes] = (payload, h)
    payload, h = _PAYLOAD[nbytes]
    f = dict(magic=b"NNLSCKP1", version=1, widths=(256, 1024, 256),
             params=int(L.nnls_mlp_param_count()), nbytes=nbytes, step=7, hash=h, reserved=0)
    f.update(over)
    head = struct.pack("<8sI3IqQqQQ", f["magic"], f["version"], *f["widths"], f["params"],
                       f["nbytes"], f["step"], f["hash"], f["reserved"])
    assert len(head) == 64
    return head + payload


def test_checkpoint_files_are_checked_before_any_device_copy(L, tmp_path):
    """nnls_mlp_load reads and checks the whole file first: every damaged or foreign file is
    refused with NNLS_E_IO before the (never dereferenced) device pointer is touched."""
    from paper_1502_01645_amd import nnls as N
    step = ctypes.c_int64(-1)
    good = _checkpoint_bytes(L)
    nbytes = int(L.nnls_mlp_blob_bytes())
    cases = {
        "missing": None,
        "empty": b"",
        "header only": good[:64],
        "truncated": good[:-1],
        "trailing byte": good + b"\0",
        "magic": _checkpoint_bytes(L, magic=b"NNLSCKP2"),
        "version": _checkpoint_bytes(L, version=2),
        "widths": _checkpoint_bytes(L, widths=(256, 512, 256)),
        "params": _checkpoint_bytes(L, params=12),
        "size field": _checkpoint_bytes(L, nbytes=nbytes - 4),
        "negative step": _checkpoint_bytes(L, step=-1),
        "hash": good[:100] + bytes([good[100] ^ 1]) + good[101:],
    }
    for name, data in cases.items():
        path = tmp_path / f"{name.replace(' ', '_')}.ckpt"
        if data is not None:
            path.write_bytes(data)
        rc = L.nnls_mlp_load(FAKE, ctypes.byref(step), os.fsencode(path), None)
        assert rc == N.E_IO, name
        assert step.value == -1, name
    # argument errors
    p = os.fsencode(tmp_path / "x.ckpt")
    assert L.nnls_mlp_load(None, None, p, None) == N.E_ARG
    assert L.nnls_mlp_load(FAKE, None, None, None) == N.E_ARG
    assert L.nnls_mlp_save(FAKE, 0, None, None) == N.E_ARG
    assert L.nnls_mlp_save(None, 0, p, None) == N.E_ARG
    assert L.nnls_mlp_save(FAKE, -1, p, None) == N.E_ARG
    # an unwritable destination is found before the device copy
    assert L.nnls_mlp_save(FAKE, 0, os.fsencode(tmp_path / "no" / "dir" / "x.ckpt"),
                           None) == N.E_IO
