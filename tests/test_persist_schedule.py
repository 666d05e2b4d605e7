"""CPU replay of the persistent batched executor's schedule
(psvt_batched_check_schedule, no device): for the batched recipe's shapes,
the small case and batches with invalid descriptors, under every schedule,
tickets map one to one onto items in (launch, matrix, item) order, each
item's dependency count is its matrix's items of earlier launches, and
simulated blocks that take tickets in order and run items for random times
drain every ticket, no item starting before its matrix's earlier launches
completed."""
import math

import numpy as np
import pytest

import paper_2607_22484_amd as psvt

SCHEDULES = [dict(), dict(n_bf16=18), dict(n_fp8=6, n_bf16=12), dict(n_bf16=18, flags=psvt.FLAG_HFORM),
             dict(n_bf16=20)]


@pytest.fixture(scope="module")
def lib():
    try:
        return psvt.load()
    except Exception as e:  # the library must be built first
        pytest.skip("libpsvt.so not built: %s" % e)


def _recipe_shapes(count, lo=128, hi=2048, seed=0):
    rng = np.random.default_rng(seed)
    sh = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=(count, 2)))).astype(int)
    return [(int(m), int(n)) for m, n in sh]


@pytest.mark.parametrize("sched", SCHEDULES, ids=["fp32", "bf16", "fp8", "hform", "split_all"])
def test_schedule_of_uneven_batch(lib, sched):
    shapes = _recipe_shapes(96, seed=1)
    tickets = psvt.check_persistent_schedule(shapes, 2048, 2048, iters=20, blocks=512, seed=3, **sched)
    assert tickets > 0


def test_schedule_of_full_recipe(lib):
    shapes = _recipe_shapes(512)
    assert psvt.check_persistent_schedule(shapes, 2048, 2048, iters=20, n_bf16=18, blocks=512, seed=5) > 512


@pytest.mark.parametrize("blocks", [1, 3, 512])
def test_schedule_small_case_and_block_counts(lib, blocks):
    assert psvt.check_persistent_schedule([(256, 128)], 256, 128, iters=20, blocks=blocks, seed=blocks) > 0


def test_schedule_with_invalid_and_rank_r(lib):
    shapes = [(300, 128), (64, 64), (5000, 3), (17, 250), (1, 1)]
    assert psvt.check_persistent_schedule(shapes, 256, 256, iters=20, blocks=7) > 0
    assert psvt.check_persistent_schedule(_recipe_shapes(40, seed=2), 2048, 2048, op=psvt.OP_RANK_R,
                                          n_bf16=18, blocks=64) > 0


def test_persistent_flag_rejected_outside_batched(lib):
    import ctypes
    cfg, keep = psvt.make_config(iters=20, flags=psvt.FLAG_PERSISTENT)
    out = ctypes.c_size_t(0)
    rc = lib.psvt_workspace_bytes(psvt.OP_SVT, 64, 32, ctypes.byref(cfg), ctypes.byref(out))
    assert rc == -1
    assert b"PERSISTENT" in lib.psvt_last_error()
    # the batched workspace with the flag holds the executor's tables
    plain, _ = psvt.make_config(iters=20)
    assert psvt.batched_workspace_bytes(8, 300, 200, cfg) > psvt.batched_workspace_bytes(8, 300, 200, plain)
