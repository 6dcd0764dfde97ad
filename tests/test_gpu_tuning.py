"""The sweep's launch variants (include/mdot.h, "Launch-variant tuning") compute the same values
bit for bit: 4 or 2 waves per SIMD for point costs, LDS staging on or off for FP32 costs. Checked
on fused sweeps, on short solves and in the batched engine, plus the table lookup itself."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2307_08507_amd import mdot as M  # noqa: E402
from paper_2307_08507_amd import workloads as W  # noqa: E402


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


def _cases():
    rng = np.random.default_rng(3)
    out = []
    for d in (2, 3):
        n = 1100
        XY = dev(rng.standard_normal((2 * n, d)), torch.float32)
        out.append((f"points d={d}", M.point_cost(XY, n, d, "sqeuclid"), n, XY))
    n = 3000  # 47 x 12 tiles
    C = dev(rng.random((n, n)), torch.float32)
    out.append(("dense f32", M.dense_cost(C), n, C))
    return out


def _run(ctx, desc, n):
    rng = np.random.default_rng(n)
    u = dev(rng.standard_normal(n) * 0.3 - np.log(n))
    v = dev(rng.standard_normal(n) * 0.3 - np.log(n))
    lr = torch.empty(n, dtype=torch.float64, device="cuda")
    lc = torch.empty_like(lr)
    ctx.lse2(desc, u, v, 40.0, lr, lc)
    r = dev(np.full(n, 1.0 / n))
    c = dev(np.full(n, 1.0 / n))
    uo, vo = torch.empty_like(r), torch.empty_like(r)
    res = ctx.solve(desc, r, c, 1e-4, M.default_params(gamma_f=2.0**7), uo, vo)
    return lr.cpu().numpy(), lc.cpu().numpy(), uo.cpu().numpy(), vo.cpu().numpy(), res


@pytest.mark.parametrize("case", [0, 1, 2])
def test_launch_variants_are_bit_identical(case):
    name, desc, n, keep = _cases()[case]
    ctx = M.Context(0)
    try:
        outs = []
        for occ, stage in ((4, 0), (2, 0), (4, 1), (2, 1)):
            ctx.tune_override(occ, stage)
            assert ctx.tune_variant(desc)[0] == occ
            print(f"{name}: occ={occ} stage={stage}", flush=True)
            outs.append(_run(ctx, desc, n))
        base = outs[0]
        for o in outs[1:]:
            for a, b in zip(base[:4], o[:4]):
                assert np.array_equal(a, b)
            assert (o[4].primal_cost, o[4].dual_bound, o[4].sweeps) == (base[4].primal_cost, base[4].dual_bound,
                                                                         base[4].sweeps)
    finally:
        ctx.close()


def test_engine_with_forced_variant_equals_solve():
    # the engine groups sweeps by kernel instance, the 2-waves point instance included
    C, r, c = W.grid_problem(20, "blobs", "sqeuclid", 1)
    n = r.size
    XY = dev(np.concatenate([W.grid_coords(20), W.grid_coords(20)]), torch.float32)
    desc = M.point_cost(XY, n, 2, "sqeuclid")
    rd, cd = dev(r), dev(c)
    alone = M.Context(0)
    eng = M.Context(0)
    try:
        eng.tune_override(2, -1)
        u0, v0 = torch.empty_like(rd), torch.empty_like(rd)
        ra = alone.solve(desc, rd, cd, 1e-5, M.default_params(), u0, v0)
        u1, v1 = torch.empty_like(rd), torch.empty_like(rd)
        t = eng.submit(desc, rd, cd, 1e-5, M.default_params(), u1, v1)
        rb = eng.poll(t, wait=True)
        assert torch.equal(u0, u1) and torch.equal(v0, v1)
        assert (ra.primal_cost, ra.sweeps) == (rb.primal_cost, rb.sweeps)
    finally:
        eng.close()
        alone.close()


def test_override_is_checked():
    ctx = M.Context(0)
    try:
        for occ, stage in ((3, -1), (0, 2), (8, 0)):
            with pytest.raises(M.MdotError):
                ctx.tune_override(occ, stage)
    finally:
        ctx.close()


def test_library_reads_the_committed_table():
    # every entry of paper_2307_08507_amd/tuning.json is what a context created without an
    # override reports for a cost of that type at the entry's measured size
    import json
    import os

    path = os.path.join(os.path.dirname(M.LIB_PATH), "..", "tuning.json")
    if "MDOT_TUNING" in os.environ or not os.path.exists(path):
        pytest.skip("no committed table in effect")
    table = json.load(open(path))
    ctx = M.Context(0)
    try:
        dummy = torch.zeros(8, dtype=torch.float32, device="cuda")
        for e in table:
            n = e["measured_at_n"]
            if e["code"] == "f32":
                desc = M.CostDesc(n=n, d=0, kind=M.COST_DENSE, dtype=M.DT_F32, data=dummy.data_ptr(), scale=1.0)
            else:
                kind = M.COST_POINTS_SQEUCLID if e["code"].startswith("pts_sq") else M.COST_POINTS_L1
                d = 2 if e["code"].endswith("2") else 3
                desc = M.CostDesc(n=n, d=d, kind=kind, dtype=M.DT_F32, data=dummy.data_ptr(), scale=0.0)
            assert ctx.tune_variant(desc) == (e["occ"], e["stage_min_tiles"]), e
    finally:
        ctx.close()
