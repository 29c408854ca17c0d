"""The entry point that allocates nothing (tp_run_noalloc, the library's
fixed workspace) against the caller-workspace run it varies (tp_run_ws),
bit for bit, on two calls in a row, the second with a smaller input, and
against the oracle."""
import ctypes
import sys

import numpy as np
import pytest

import synth
from helpers import oracle_run, to_genomes

pytestmark = pytest.mark.gpu

BLOCKED = 4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1602_05856_amd as tp
    tp.lib()


def same(a, b):
    return (np.array_equal(a.junction_offset, b.junction_offset) and
            np.array_equal(a.junction_pos, b.junction_pos) and
            np.array_equal(a.vertex, b.vertex) and np.array_equal(a.strand, b.strand) and
            np.array_equal(a.edges, b.edges))


def test_noalloc_equals_workspace_run_twice():
    import torch

    import paper_1602_05856_amd as tp
    big = synth.plain_small(0)
    small = [g[:30000] for g in synth.plain_small(4)[:2]]
    cases = [(big, 25, 2**24, 3, BLOCKED, 1), (small, 31, 2**20, 2, 0, 2)]
    for i, (codes, k, b, h, flags, rounds) in enumerate(cases):
        say("case: noalloc call %d, %d genomes, %d bases, k=%d flags=%d rounds=%d" % (
            i, len(codes), sum(c.size for c in codes), k, flags, rounds))
        plan = tp.Plan(to_genomes(codes), k, b, h, flags)
        plan.rounds = rounds
        d_in = plan.upload()
        L = plan.workspace_layout(1.0, 1.0)
        assert L["workspace_bytes"] <= tp.NOALLOC_WORKSPACE_MAX
        # the existing entry point on a caller workspace
        ws, out_ws = plan.alloc_workspace()
        plan.prepare_workspace(ws)
        plan.run_ws(d_in, ws, out_ws)
        # the fixed workspace: outputs poisoned first, so every word is written
        out_na = torch.full((L["output_bytes"],), 0x77, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        plan.run_noalloc(d_in, out_na)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        c_ws, c_na = plan.ws_counts(out_ws), plan.ws_counts(out_na)
        assert c_ws["status"] == 0 and c_na == c_ws
        r_ws, r_na = plan.ws_result(out_ws), plan.ws_result(out_na)
        assert same(r_ws, r_na), "fixed workspace differs from the caller workspace"
        o, junctions, vx, edges = oracle_run(codes, k, b, h, flags) if rounds == 1 else \
            (None, None, None, None)
        if junctions is not None:
            for g in range(len(codes)):
                assert np.array_equal(r_na.junctions(g), junctions[g]), g
        plan.close()


def test_noalloc_rejects_a_workspace_beyond_its_maximum():
    import paper_1602_05856_amd as tp
    codes = synth.plain_small(0)
    plan = tp.Plan(to_genomes(codes), 25, 2**30, 3, BLOCKED)  # a 128 MiB filter
    d_in = plan.upload()
    L = plan.workspace_layout(1.0, 1.0)
    assert L["workspace_bytes"] > tp.NOALLOC_WORKSPACE_MAX
    rc = tp.lib().tp_run_noalloc(plan.handle, ctypes.c_void_p(d_in.data_ptr()),
                                 ctypes.c_void_p(d_in.data_ptr()), None)
    assert rc == tp.TP_EINVAL and "fixed workspace" in tp.last_error()
    plan.close()
