"""rk_search_static (the whole search with its scratch in the library's static
device array, no allocation) against rk_count + rk_collect with caller
buffers, through the C ABI: two calls in a row, the second with a smaller
input, both integer results compared exactly."""
import ctypes

import numpy as np
import pytest

import rkgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1810_01051_amd as rk
    return rk


def static_search(ctx, plan, text, cap):
    lib = ctx.lib
    offsets = torch.full((plan.k + 1,), -1, dtype=torch.int64, device="cuda:0")
    positions = torch.full((max(cap, 1),), -1, dtype=torch.int64, device="cuda:0")
    total = ctypes.c_uint64()
    st = lib.rk_search_static(ctx.h, plan.h, ctypes.c_void_p(text.data_ptr()), text.numel(),
                              ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(positions.data_ptr()), cap,
                              ctypes.byref(total), None)
    torch.cuda.synchronize()
    return st, int(total.value), offsets, positions


@pytest.mark.parametrize("mode", ["screen", "exact"])
def test_static_search_matches_caller_buffers(rk, mode):
    ctx = rk.Context(0)
    try:
        big = rkgen.config3(n=(1 << 22) + 11, k=200, sampled=120)
        small = rkgen.config3(n=(1 << 20) + 3, k=40, sampled=30)
        for case in (big, small):
            text = torch.from_numpy(case.text).to("cuda:0")
            plan = rk.Plan(ctx, case.patterns, mode)
            ro, rp = plan.search(text)
            torch.cuda.synchronize()
            ref_total = int(ro[-1])
            st, total, off, pos = static_search(ctx, plan, text, ref_total)
            assert st == 0, ctx.lib.rk_ctx_last_error(ctx.h)
            assert total == ref_total > 300
            assert torch.equal(off, ro)
            assert torch.equal(pos[:total], rp[:total])
            # one pattern: the single-bucket kernel
            p1 = rk.Plan(ctx, case.patterns[:1], mode)
            o1, q1 = p1.search(text)
            st, t1, off1, pos1 = static_search(ctx, p1, text, int(o1[-1]))
            assert st == 0 and t1 == int(o1[-1])
            assert torch.equal(off1, o1) and torch.equal(pos1[:t1], q1[:t1])
            p1.close()
            plan.close()
    finally:
        ctx.close()


def test_static_search_rejects_oversize(rk):
    ctx = rk.Context(0)
    try:
        lib = ctx.lib
        limit = lib.rk_static_scratch_bytes()
        assert limit > 0
        text = torch.zeros(1 << 30, dtype=torch.uint8, device="cuda:0")
        plan = rk.Plan(ctx, [b"xyz"], "screen")
        st, total, _, _ = static_search(ctx, plan, text, 16)
        assert st == rk._lib.RK_ENOSPACE
        assert b"static array" in ctx.lib.rk_ctx_last_error(ctx.h)
        # capacity below the total: RK_ENOSPACE after the count, total reported
        g = rkgen.rng(60, 0)
        t2 = torch.from_numpy(rkgen.iid_text(g, 1 << 16, rkgen.ACGT)).to("cuda:0")
        p2 = rk.Plan(ctx, [b"A"], "screen")
        st, total, _, _ = static_search(ctx, p2, t2, 10)
        assert st == rk._lib.RK_ENOSPACE and total > 10
        p2.close()
        plan.close()
    finally:
        ctx.close()
