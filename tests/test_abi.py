"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2607_22484_amd as psvt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "psvt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(psvt_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported():
    lib = psvt.load()
    names = header_symbols()
    assert names, "no declarations found"
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(psvt.EXPORTED) == names


def test_strerror_and_version():
    lib = psvt.load()
    assert lib.psvt_strerror(0) == b"success"
    assert lib.psvt_strerror(psvt.PSVT_EWORKSPACE).startswith(b"workspace")
    assert b"gfx950" in lib.psvt_version()


def test_workspace_bytes():
    n1 = psvt.workspace_bytes(psvt.OP_SVT, 256, 128)
    n2 = psvt.workspace_bytes(psvt.OP_SVT, 4096, 4096)
    assert 0 < n1 < n2
    assert psvt.workspace_bytes(psvt.OP_SVT, 0, 5) == 0
    # left- and right-sided plans of transposed shapes need the same space
    assert psvt.workspace_bytes(psvt.OP_SVT, 300, 200) == psvt.workspace_bytes(psvt.OP_SVT, 200, 300)
    assert psvt.workspace_bytes(psvt.OP_RANK_R, 512, 512) < psvt.workspace_bytes(psvt.OP_SVT, 512, 512)
    with pytest.raises(psvt.PsvtError):
        psvt.workspace_bytes(psvt.OP_POLAR_SYM, 5, 6)
    with pytest.raises(psvt.PsvtError):
        psvt.workspace_bytes(9, 5, 6)


def batch_ws(m, n, cfg):
    lib = psvt.load()
    items = (psvt.BatchItem * 1)()
    items[0] = psvt.BatchItem(1 << 40, 1 << 41, m, n, n, n, 0.5)
    out = ctypes.c_size_t(0)
    assert lib.psvt_batch_workspace_bytes(psvt.OP_SVT, items, 1, ctypes.byref(cfg), ctypes.byref(out)) == 0
    return out.value


@pytest.mark.parametrize("m,n", [(300, 200), (2048, 3000), (3000, 2049)])
def test_workspace_fork_copies(m, n):
    """A single low-precision call with min(m, n) <= 2048 runs P's iterations
    on a side stream and needs two more s x s copies (X^2 and B of S); batch
    items, FP32 schedules and larger s share them."""
    s = min(m, n)
    ld = -(-s // 64) * 64
    extra = 2 * (-(-4 * s * ld // 256) * 256)
    fp32, _ = psvt.make_config(iters=20)
    bf16, _ = psvt.make_config(iters=20, n_bf16=18)
    assert psvt.workspace_bytes(psvt.OP_SVT, m, n, fp32) == batch_ws(m, n, fp32)
    fork = s <= 2048
    assert psvt.workspace_bytes(psvt.OP_SVT, m, n, bf16) == batch_ws(m, n, bf16) + (extra if fork else 0)


FAKE = ctypes.c_void_p(1 << 40)  # never dereferenced: every call below fails validation first


def call_svt(m=8, n=4, lda=4, tau=0.5, Y=FAKE, ldy=4, ws=FAKE, ws_bytes=1 << 30, cfg=None, A=FAKE):
    lib = psvt.load()
    return lib.psvt_svt(A, m, n, lda, tau, Y, ldy, ws, ws_bytes, ctypes.byref(cfg) if cfg else None, None)


@pytest.mark.parametrize("kw", [
    dict(lda=3), dict(ldy=2), dict(tau=-1.0), dict(tau=float("nan")), dict(tau=float("inf")),
    dict(A=None), dict(Y=None), dict(m=-1),
])
def test_svt_rejects_bad_arguments(kw):
    assert call_svt(**kw) == psvt.PSVT_EINVAL
    assert psvt.load().psvt_last_error()


def test_svt_workspace_errors():
    assert call_svt(ws=None) == psvt.PSVT_EWORKSPACE
    assert call_svt(ws_bytes=16) == psvt.PSVT_EWORKSPACE
    assert call_svt(ws=ctypes.c_void_p((1 << 40) + 8)) == psvt.PSVT_EINVAL  # misaligned


def test_svt_rejects_overlap():
    # Y inside the workspace range
    assert call_svt(Y=ctypes.c_void_p((1 << 40) + 4096)) == psvt.PSVT_EINVAL


def test_config_validation():
    cfg, _ = psvt.make_config(iters=300)
    assert call_svt(cfg=cfg) == psvt.PSVT_EINVAL
    cfg, _ = psvt.make_config(iters=4, n_bf16=3, n_fp8=2)
    assert call_svt(cfg=cfg) == psvt.PSVT_EINVAL
    cfg, _ = psvt.make_config(side=7)
    assert call_svt(cfg=cfg) == psvt.PSVT_EINVAL
    cfg, keep = psvt.make_config(iters=2, coeffs=[1.0, 0.0, float("nan"), 1, 0, 0])
    assert call_svt(cfg=cfg) == psvt.PSVT_EINVAL
    cfg, _ = psvt.make_config(flags=0x80)            # unknown flag
    assert call_svt(cfg=cfg) == psvt.PSVT_EINVAL
    cfg, _ = psvt.make_config(flags=psvt.FLAG_SPLIT_P | psvt.FLAG_PLAIN_P)
    assert call_svt(cfg=cfg) == psvt.PSVT_EINVAL
    cfg, _ = psvt.make_config(flags=psvt.FLAG_STATUS)  # status flag without a status word
    assert call_svt(cfg=cfg) == psvt.PSVT_EINVAL
    for safety in (0.5, 17.0, float("nan")):
        cfg, _ = psvt.make_config(norm_safety=safety)
        assert call_svt(cfg=cfg) == psvt.PSVT_EINVAL
    for tol in (-1.0, float("inf")):
        cfg, _ = psvt.make_config(status=1 << 40, status_tol=tol)
        assert call_svt(cfg=cfg) == psvt.PSVT_EINVAL
    cfg, _ = psvt.make_config(flags=psvt.FLAG_HFORM)
    assert psvt.load().psvt_rank_r(FAKE, 8, 4, 4, 0.5, FAKE, 4, FAKE, 1 << 30, ctypes.byref(cfg), None) == psvt.PSVT_EINVAL
    lib = psvt.load()
    apart = dict(A=ctypes.c_void_p(1 << 43), Y=ctypes.c_void_p(1 << 41))  # A, Y and ws apart
    cfg, _ = psvt.make_config(warm_iters=65)
    assert call_svt(cfg=cfg, **apart) == psvt.PSVT_EINVAL and b"warm_iters" in lib.psvt_last_error()
    cfg, _ = psvt.make_config()
    cfg.warm_pi, cfg.ld_pi = 1 << 42, 2       # ld_pi below the Gram side (4)
    assert call_svt(cfg=cfg, **apart) == psvt.PSVT_EINVAL and b"ld_pi" in lib.psvt_last_error()
    cfg.warm_pi, cfg.ld_pi = (1 << 40) + 256, 4  # inside ws
    assert call_svt(cfg=cfg, **apart) == psvt.PSVT_EINVAL and b"overlap ws" in lib.psvt_last_error()
    cfg.warm_pi, cfg.ld_pi, cfg.warm_iters = 1 << 42, 4, 1   # a warm start needs at least 2 steps
    assert call_svt(cfg=cfg, **apart) == psvt.PSVT_EINVAL and b"warm_iters" in lib.psvt_last_error()
    cfg, _ = psvt.make_config(n_fp8=2, flags=psvt.FLAG_HFORM)
    assert call_svt(cfg=cfg, **apart) == psvt.PSVT_EINVAL and b"HFORM" in lib.psvt_last_error()
    # accepted settings reach the workspace check (ws = NULL here)
    for kw in (dict(flags=psvt.FLAG_PLAIN_P), dict(norm_safety=1.5), dict(status=1 << 40, status_tol=1e-4)):
        cfg, _ = psvt.make_config(**kw)
        assert call_svt(cfg=cfg, ws=None) == psvt.PSVT_EWORKSPACE, kw


def test_config_struct_layout():
    """The binding's Config mirrors psvt_config (size and field offsets as a
    C compiler lays them out)."""
    import subprocess
    import tempfile
    src = (b'#include <stddef.h>\n#include <stdio.h>\n#include "psvt.h"\nint main(void){printf("%zu %zu %zu %zu %zu'
           b' %zu %zu %zu %zu %zu %zu %zu\\n",'
           b' sizeof(psvt_config), offsetof(psvt_config, flags), offsetof(psvt_config, norm_safety),'
           b' offsetof(psvt_config, status), offsetof(psvt_config, status_tol), offsetof(psvt_config, warm_pi),'
           b' offsetof(psvt_config, ld_pi), offsetof(psvt_config, warm_iters), sizeof(psvt_batch_item),'
           b' offsetof(psvt_batch_item, warm_pi), offsetof(psvt_batch_item, ld_pi), sizeof(psvt_desc));'
           b' return 0;}\n')
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        with open(c, "wb") as f:
            f.write(src)
        exe = os.path.join(d, "l")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        got = [int(x) for x in subprocess.check_output([exe]).split()]
    C, B = psvt.Config, psvt.BatchItem
    assert got == [ctypes.sizeof(C), C.flags.offset, C.norm_safety.offset, C.status.offset, C.status_tol.offset,
                   C.warm_pi.offset, C.ld_pi.offset, C.warm_iters.offset, ctypes.sizeof(B), B.warm_pi.offset,
                   B.ld_pi.offset, ctypes.sizeof(psvt.Desc)]


def test_noalloc_rejects_sizes_beyond_its_scratch():
    """psvt_svt_noalloc refuses, before touching the device, a problem whose
    workspace exceeds the static scratch (4096^2 needs ~0.9 GB)."""
    lib = psvt.load()
    rc = lib.psvt_svt_noalloc(FAKE, 4096, 4096, 4096, 0.5, ctypes.c_void_p(1 << 41), 4096, None, None)
    assert rc == psvt.PSVT_EWORKSPACE
    assert b"PSVT_NOALLOC_SCRATCH_BYTES" in lib.psvt_last_error()
    cfg, _ = psvt.make_config(iters=300)
    assert lib.psvt_svt_noalloc(FAKE, 8, 4, 4, 0.5, FAKE, 4, ctypes.byref(cfg), None) == psvt.PSVT_EINVAL
    assert lib.psvt_svt_noalloc(None, 0, 4, 4, 0.5, None, 4, None, None) == psvt.PSVT_OK


def test_empty_is_noop():
    # m == 0 returns before any pointer is used
    assert call_svt(m=0, A=None, Y=None, ws=None) == psvt.PSVT_OK


def test_other_entry_points_validate():
    lib = psvt.load()
    assert lib.psvt_polar(FAKE, 5, 4, 3, FAKE, 4, FAKE, 1 << 30, None, None) == psvt.PSVT_EINVAL
    assert lib.psvt_polar_sym(FAKE, 5, 4, FAKE, 5, FAKE, 1 << 30, None, None) == psvt.PSVT_EINVAL
    assert lib.psvt_rank_r(FAKE, 5, 4, 4, -0.1, FAKE, 4, FAKE, 1 << 30, None, None) == psvt.PSVT_EINVAL
    assert lib.psvt_gemm_nt(0, FAKE, 4, FAKE, 4, None, 0, FAKE, 4, 3, 4, 4, 1.0, 0.0, 1, None) == psvt.PSVT_EINVAL
    assert lib.psvt_gemm_nt(0, ctypes.c_void_p((1 << 40) + 4), 4, FAKE, 4, None, 0, FAKE, 4, 4, 4, 4, 1.0, 0.0, 0,
                            None) == psvt.PSVT_EINVAL
    assert lib.psvt_gemm_nt(1, FAKE, 4, FAKE, 8, None, 0, FAKE, 4, 4, 4, 4, 1.0, 0.0, 0, None) == psvt.PSVT_EINVAL
    assert lib.psvt_gemm_nt(5, FAKE, 4, FAKE, 4, None, 0, FAKE, 4, 4, 4, 4, 1.0, 0.0, 0, None) == psvt.PSVT_EINVAL
    assert lib.psvt_convert(1, FAKE, 4, 4, 3, FAKE, 4, 1.0, 0, None) == psvt.PSVT_EINVAL
    assert lib.psvt_convert(9, FAKE, 4, 4, 4, FAKE, 4, 1.0, 0, None) == psvt.PSVT_EINVAL


def test_python_wrapper_rejects_non_2d():
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError):
        psvt.svt(torch.zeros(2, 3, 4), 0.1)
    with pytest.raises(TypeError):
        psvt.svt(torch.zeros(3, 4, dtype=torch.float64), 0.1)
    with pytest.raises(TypeError):
        psvt.svt(torch.zeros(3, 4), 0.1)  # CPU tensor


def test_tune_table_parsing(tmp_path):
    lib = psvt.load()
    good = tmp_path / "good.txt"
    good.write_text("# comment\n0 1 0 0.5 10\n\n1 3 1 0.7 5.5  # trailing\n")
    assert lib.psvt_tune_load(str(good).encode()) == psvt.PSVT_OK
    for text in ["0 1 0 0.5\n", "0 5 0 0.5 1\n", "0 1 2 0.5 1\n", "0 1 0 1.5 1\n", "0 1 0 0.5 -1\n",
                 "0 1 0 0.5 1 extra\n", "4 1 0 0.5 1\n"]:
        bad = tmp_path / "bad.txt"
        bad.write_text(text)
        assert lib.psvt_tune_load(str(bad).encode()) == psvt.PSVT_EINVAL, text
    assert lib.psvt_tune_load(str(tmp_path / "missing.txt").encode()) == psvt.PSVT_EINVAL
    # restore the shipped table
    if os.path.exists(psvt.TUNE_TABLE):
        assert lib.psvt_tune_load(psvt.TUNE_TABLE.encode()) == psvt.PSVT_OK


def test_tune_pick_model():
    """The cost model: a full 4096 product fits one round of 256x256 tiles or
    two of 128x128; a symmetric 4096 product (lower triangle) fits one round
    of 192 tiles (528 tiles of 128 would need a second round);
    small products use the 64 tiles (more blocks)."""
    lib = psvt.load()
    assert lib.psvt_tune_load(psvt.TUNE_TABLE.encode()) == psvt.PSVT_OK
    assert psvt.pick_tile(4096, 4096, 4096, True) == psvt.TILE_IDS[192]
    assert psvt.pick_tile(4096, 4096, 4096, False) in (psvt.TILE_IDS[128], psvt.TILE_IDS[256])
    assert psvt.pick_tile(4096, 4096, 4096, True, dtype=psvt.DTYPE_BF16) == psvt.TILE_IDS[192]
    assert psvt.pick_tile(512, 512, 512, True) == psvt.TILE_IDS[64]
    assert lib.psvt_tune_pick(0, 0, 5, 5, 0) == psvt.PSVT_EINVAL
    assert lib.psvt_tune_pick(7, 5, 5, 5, 0) == psvt.PSVT_EINVAL
    assert lib.psvt_tune_force_tile(9) == psvt.PSVT_EINVAL
    assert lib.psvt_tune_set(0, 1, 0, 0.0, 1.0) == psvt.PSVT_EINVAL


def test_batch_validation():
    lib = psvt.load()
    items = (psvt.BatchItem * 2)()
    items[0] = psvt.BatchItem(1 << 40, 1 << 41, 8, 4, 4, 4, 0.5)
    items[1] = psvt.BatchItem(1 << 40, 1 << 41, 8, 4, 3, 4, 0.5)   # lda < n
    out = ctypes.c_size_t(0)
    assert lib.psvt_batch_workspace_bytes(0, items, 2, None, ctypes.byref(out)) == psvt.PSVT_EINVAL
    assert lib.psvt_batch_workspace_bytes(0, items, 1, None, ctypes.byref(out)) == psvt.PSVT_OK
    assert out.value == psvt.workspace_bytes(psvt.OP_SVT, 8, 4)
    assert lib.psvt_batch_workspace_bytes(1, items, 1, None, ctypes.byref(out)) == psvt.PSVT_EINVAL  # polar
    assert lib.psvt_batch_workspace_bytes(0, items, 0, None, ctypes.byref(out)) == psvt.PSVT_EINVAL
    h = ctypes.c_void_p()
    assert lib.psvt_batch_create(0, items, 1, None, 1 << 30, None, ctypes.byref(h)) == psvt.PSVT_EWORKSPACE
    assert lib.psvt_batch_run(None, None) == psvt.PSVT_EINVAL
    assert lib.psvt_batch_destroy(None) == psvt.PSVT_OK


def test_batched_device_descriptors_validate():
    """psvt_svt_batched checks count, maxima, configuration and workspace on
    the host before any launch; its stage template relocates for every
    schedule, side and flag set (the self-check on probe matrices runs
    before the workspace check, so EWORKSPACE means it passed)."""
    lib = psvt.load()
    out = ctypes.c_size_t(0)
    assert lib.psvt_batched_workspace_bytes(0, -1, 8, 8, None, ctypes.byref(out)) == psvt.PSVT_EINVAL
    assert lib.psvt_batched_workspace_bytes(0, 4, 0, 8, None, ctypes.byref(out)) == psvt.PSVT_EINVAL
    assert lib.psvt_batched_workspace_bytes(1, 4, 8, 8, None, ctypes.byref(out)) == psvt.PSVT_EINVAL  # polar
    assert lib.psvt_batched_workspace_bytes(0, 0, 8, 8, None, ctypes.byref(out)) == psvt.PSVT_OK and out.value == 0
    assert lib.psvt_batched_workspace_bytes(0, 3, 300, 200, None, ctypes.byref(out)) == psvt.PSVT_OK
    assert out.value >= 3 * psvt.workspace_bytes(psvt.OP_SVT, 300, 200)
    assert lib.psvt_svt_batched(FAKE, 0, 8, 8, None, 0, None, None) == psvt.PSVT_OK         # empty batch
    assert lib.psvt_svt_batched(None, 2, 8, 8, FAKE, 1 << 30, None, None) == psvt.PSVT_EINVAL
    schedules = [dict(), dict(n_bf16=18), dict(n_fp8=6, n_bf16=12), dict(n_bf16=20),
                 dict(n_bf16=18, flags=psvt.FLAG_PLAIN_P), dict(n_bf16=18, flags=psvt.FLAG_PLAIN_S),
                 dict(flags=psvt.FLAG_STATUS), dict(n_bf16=18, flags=psvt.FLAG_STATUS), dict(iters=1),
                 dict(iters=7, n_fp8=3), dict(side=psvt.SIDE_LEFT), dict(side=psvt.SIDE_RIGHT, n_bf16=4),
                 dict(norm_safety=2.0), dict(n_bf16=18, flags=psvt.FLAG_HFORM),
                 dict(n_bf16=12, flags=psvt.FLAG_HFORM | psvt.FLAG_STATUS)]
    for kw in schedules:
        cfg, _ = psvt.make_config(**kw)
        for entry in (lib.psvt_svt_batched, lib.psvt_rank_r_batched):
            rc = entry(FAKE, 2, 64, 48, FAKE, 1024, ctypes.byref(cfg), None)
            if entry is lib.psvt_rank_r_batched and kw.get("flags", 0) & psvt.FLAG_HFORM:
                assert rc == psvt.PSVT_EINVAL   # the H-form needs the polar factor: svt only
            else:
                assert rc == psvt.PSVT_EWORKSPACE, (kw, lib.psvt_last_error())


def test_tune_model_replica_matches_library_picks():
    """The tuner's replica of the cost model (used to refit and report
    regret off the device) picks what the library picks for the committed
    table, over random product shapes of every operand type; the committed
    table has no efficiency clamped at 1."""
    from paper_2607_22484_amd import tune
    lib = psvt.load()
    assert lib.psvt_tune_load(psvt.TUNE_TABLE.encode()) == psvt.PSVT_OK
    table = {}
    with open(psvt.TUNE_TABLE) as f:
        for line in f:
            line = line.split("#")[0].split()
            if line:
                dt, t, sym, e, o = int(line[0]), int(line[1]), int(line[2]), float(line[3]), float(line[4])
                table[(dt, t, sym)] = (e, o)
    assert len(table) == 32 and all(0.0 < e < 1.0 for e, _ in table.values())
    rng = np.random.default_rng(7)
    for _ in range(400):
        dt = int(rng.integers(0, 4))
        sym = bool(rng.integers(0, 2))
        M = int(rng.integers(1, 9000))
        N = M if sym else int(rng.integers(1, 9000))
        K = int(rng.integers(1, 9000))
        assert psvt.pick_tile(M, N, K, sym, dt) == tune.model_pick(table, dt, M, N, K, sym), (dt, M, N, K, sym)
