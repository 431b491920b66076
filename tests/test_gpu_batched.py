"""Uneven batch (one captured graph over many independent problems) against the FP64 oracle,
with the default per-class parameters, with every Gram tile size and solver workgroup size set
through a tuning cache, and with the parameters nnls_autotune measures."""
import json

import numpy as np
import pytest
import torch

from gpu_common import DEV, gram_abs_tol, host, orc, say
from oracle import oracle as O
from paper_1502_01645_amd import nnls as N
from paper_1502_01645_amd import workloads as W

pytestmark = pytest.mark.gpu


def _problems():
    """Edge sizes around the 128-wide tiles and the 64-entry ownership chunks, plus problems
    of the batched workload recipe (n ~ U{16..512}, d = 3n)."""
    rng = np.random.default_rng(51)
    probs = []
    for n, d in [(1, 3), (2, 6), (7, 21), (16, 48), (63, 189), (64, 64), (65, 195), (127, 381),
                 (128, 128), (129, 387), (255, 300), (256, 768), (257, 771), (384, 1152)]:
        A = rng.random((d, n)).astype(np.float32)
        x = np.where(rng.random(n) < 0.6, 0.0, rng.random(n))
        b = (A.astype(np.float64) @ x + 0.01 * rng.standard_normal(d)).astype(np.float32)
        probs.append((A, b))
    for i in range(10):
        A, b, _ = W.make_batched_problem(i)
        probs.append((A, b[:, 0]))
    return probs


@pytest.fixture(scope="module")
def solved():
    probs = _problems()
    say(f"batched plan over {len(probs)} problems")
    A_pool, B_pool, descs = N.pack_problems(probs, DEV)
    plan = N.BatchedPlan(A_pool, B_pool, descs, tol=3e-6, max_iter=100000)
    plan.launch()
    torch.cuda.synchronize()
    return probs, plan


def test_batched_rescaled_problem(solved):
    probs, plan = solved
    Qp = host(plan.Q_pool)
    qp = host(plan.q_pool)
    for i, (A, b) in enumerate(probs):
        dsc = plan.descs[i]
        n, d = dsc.n, dsc.d
        Q = Qp[dsc.offQ:dsc.offQ + n * n].reshape(n, n).astype(np.float64)
        s_o, Q_o, q_o = orc().prepare(A, b.reshape(-1, 1))
        # the batch takes its scales from the computed Gram diagonal: any positive scaling is
        # an exact rescale, so Q still matches the cosine matrix within the Gram error (x2 for
        # the scale error)
        tol = 2 * gram_abs_tol(d, "bf16x3")
        assert np.abs(Q - Q_o).max() <= tol, (i, np.abs(Q - Q_o).max())
        assert np.array_equal(Q, Q.T)
        assert np.all(np.diag(Q) == 1.0)
        q = qp[dsc.offq:dsc.offq + n].astype(np.float64)
        assert np.abs(q - q_o[:, 0]).max() <= tol * np.linalg.norm(b), i


def test_batched_solutions_meet_tolerances(solved):
    probs, plan = solved
    st = host(plan.status)
    assert np.all(st == N.CONVERGED), st
    X = host(plan.X_pool)
    worst_r, worst_gap = 0.0, 0.0
    for i, (A, b) in enumerate(probs):
        dsc = plan.descs[i]
        x = X[dsc.offX:dsc.offX + dsc.n].reshape(-1, 1)
        assert np.all(x >= 0)
        r, F = orc().kkt_x(A, b.reshape(-1, 1), x)
        ref = O.reference_solution(A, b.reshape(-1, 1))
        gap = O.relative_gap(F, ref)
        worst_r, worst_gap = max(worst_r, r[0]), max(worst_gap, gap[0])
        assert r[0] <= 1e-5, (i, dsc.n, r[0])
        assert gap[0] <= 1e-6, (i, dsc.n, gap[0])
    say(f"batched: worst r={worst_r:.3e} worst gap={worst_gap:.3e}")


def test_batched_graph_replays_identical(solved):
    """Relaunching the captured graph (with eager work in between) reproduces every output."""
    probs, plan = solved
    X0, it0 = host(plan.X_pool).copy(), host(plan.iters).copy()
    for rep in range(3):
        junk = torch.randn(1 << 20, device=DEV)
        junk.mul_(2.0).sum()
        torch.cuda.synchronize()
        plan.X_pool.fill_(-1.0)
        plan.launch()
        torch.cuda.synchronize()
        assert np.array_equal(host(plan.X_pool), X0), rep
        assert np.array_equal(host(plan.iters), it0), rep


def test_batched_matches_per_problem_launches(solved):
    """The batch gives the same quality as solving each problem with its own C-ABI calls."""
    probs, plan = solved
    for i in [0, 5, 9, 13, 20]:
        A, b = probs[i]
        res = N.nnls(torch.from_numpy(A).to(DEV), torch.from_numpy(b.reshape(-1, 1)).to(DEV),
                     tol=1e-5, max_iter=100000, inner_tol=3e-6, refine_step=False)
        r1, _ = orc().kkt_x(A, b.reshape(-1, 1), host(res["X"]))
        assert r1[0] <= 1e-5


# every size class present in _problems(): n <= 64, 128, 256, 512
# (gram tile, solver workgroup threads, resident workgroups per compute unit: 0 = all that fit)
_FORCED = {(1, 64): (64, 1024, 0), (65, 128): (64, 512, 1), (129, 256): (128, 1024, 1),
           (257, 512): (64, 256, 0)}


def _write_cache(path, params):
    import torch as _t
    arch = _t.cuda.get_device_properties(0).gcnArchName
    lines = [json.dumps({"arch": arch, "op": "batched", "dtype": "f32", "n_lo": lo, "n_hi": hi,
                         "gram_tile": t, "solve_threads": nt, "solve_wgs_per_cu": pc})
             for (lo, hi), (t, nt, pc) in params.items()]
    with open(path, "w") as f:
        f.write('{"format": "nnls-autotune-1", "entries": [\n' + ",\n".join(lines) + "\n]}\n")


def _check_plan(probs, plan, ref_plan):
    """Same Gram as the default plan bit for bit (a Gram entry's sum over d does not depend on
    the tile size), every problem converged and within the tolerances against the oracle."""
    assert np.array_equal(host(plan.Q_pool), host(ref_plan.Q_pool))
    assert np.array_equal(host(plan.q_pool), host(ref_plan.q_pool))
    assert np.array_equal(host(plan.s_pool), host(ref_plan.s_pool))
    assert np.all(host(plan.status) == N.CONVERGED)
    X = host(plan.X_pool)
    for i, (A, b) in enumerate(probs):
        dsc = plan.descs[i]
        x = X[dsc.offX:dsc.offX + dsc.n].reshape(-1, 1)
        r, F = orc().kkt_x(A, b.reshape(-1, 1), x)
        gap = O.relative_gap(F, O.reference_solution(A, b.reshape(-1, 1)))
        assert r[0] <= 1e-5 and gap[0] <= 1e-6, (i, dsc.n, r[0], gap[0])


def test_batched_every_tile_and_workgroup_size(solved, tmp_path):
    """A cache that sets 64-wide Gram tiles and 512- and 1024-thread solver workgroups for some
    classes: the plan reads it and every kernel variant gives the default plan's Gram and
    solutions within the tolerances."""
    probs, ref = solved
    path = str(tmp_path / "forced.json")
    _write_cache(path, _FORCED)
    A_pool, B_pool, descs = N.pack_problems(probs, DEV)
    plan = N.BatchedPlan(A_pool, B_pool, descs, tol=3e-6, max_iter=100000, tune_cache=path)
    plan.launch()
    torch.cuda.synchronize()
    _check_plan(probs, plan, ref)
    # replays of the captured graph are deterministic
    X0 = host(plan.X_pool).copy()
    plan.launch()
    torch.cuda.synchronize()
    assert np.array_equal(host(plan.X_pool), X0)


def test_autotune_writes_cache_the_plan_uses(solved, tmp_path):
    """nnls_autotune through the C ABI on the shapes of the batch: the cache is JSON with one
    entry per size class present (measured times for every candidate, the fastest chosen), a
    second call keeps the entries of other keys, and a plan built from the cache solves the
    batch within the tolerances."""
    probs, ref = solved
    path = str(tmp_path / "tune.json")
    shapes = [(A.shape[0], A.shape[1]) for A, _ in probs]
    say(f"autotune over {len(shapes)} shapes")
    N.autotune(path, shapes)
    with open(path) as f:
        cache = json.load(f)
    entries = cache["entries"]
    say("  " + "; ".join(f"n<={e['n_hi']}: tile {e['gram_tile']} threads {e['solve_threads']}"
                         f" per CU {e['solve_wgs_per_cu']}" for e in entries))
    assert sorted((e["n_lo"], e["n_hi"]) for e in entries) == sorted(_FORCED)
    for e in entries:
        assert e["op"] == "batched" and e["dtype"] == "f32"
        assert e["gram_tile"] in (64, 128) and e["solve_threads"] in (256, 512, 1024)
        assert e["solve_wgs_per_cu"] in (0, 1)
        gm, sm = e["gram_ms"], e["solve_ms"]
        assert e["gram_tile"] == min((64, 128), key=lambda t: gm[str(t)])
        chosen = f"{e['solve_threads']}" + ("/1" if e["solve_wgs_per_cu"] else "")
        assert len(sm) == 6 and sm[chosen] == min(sm.values())
        assert all(v > 0 for v in list(gm.values()) + list(sm.values()))
    # a second tuning of one class replaces only that class's entry
    N.autotune(path, [s for s in shapes if s[1] <= 64])
    with open(path) as f:
        again = json.load(f)["entries"]
    assert sorted((e["n_lo"], e["n_hi"]) for e in again) == sorted(_FORCED)
    A_pool, B_pool, descs = N.pack_problems(probs, DEV)
    plan = N.BatchedPlan(A_pool, B_pool, descs, tol=3e-6, max_iter=100000, tune_cache=path)
    plan.launch()
    torch.cuda.synchronize()
    _check_plan(probs, plan, ref)
