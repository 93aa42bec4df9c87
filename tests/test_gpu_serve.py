"""The continuous-batching request loop: requests of several classes arrive
over time and share one HBM budget (here too small to hold them all at
once): they are admitted as room frees up, pools grow and give back slots,
moving their members, and every result equals the same request solved
alone (bitwise: the pool runs the same kernels as a single forest with the
pool's default stage kernel)."""
import numpy as np
import pytest

from paper_2502_12620_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _requests():
    rng = np.random.default_rng(7)
    out = []
    t = 0.0
    for i in range(14):
        t += float(rng.exponential(0.002))
        dim = 2 if i % 3 else 3
        p = int(rng.integers(1, 4))
        steps = int(rng.integers(2, 7))
        if dim == 2:
            roots = (int(rng.integers(1, 4)), int(rng.integers(1, 4)))
            L = (2.5 * roots[0], 2.5 * roots[1])
            w = W.Workload(f"r{i}", 2, p, 8, roots, (0.0, 0.0), L, (W.PERIODIC,) * 2, 1, W.IC_VORTEX,
                           [3.0, L[0] / 2, L[1] / 2, 1.0, 1.0, L[0], L[1]], steps, cfl=0.05 + 0.05 * (i % 3))
        else:
            roots = (int(rng.integers(1, 3)), 2, 1)
            L = (1.25 * roots[0], 2.5, 1.25)
            w = W.Workload(f"r{i}", 3, p, 4, roots, (0.0,) * 3, L, (W.PERIODIC,) * 3, 1, W.IC_VORTEX,
                           [3.0, L[0] / 2, L[1] / 2, 1.0, 1.0, L[0], L[1]], steps)
        out.append((t, w))
    return out


def _alone(w):
    from paper_2502_12620_amd import dgamr as G

    f = G.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma)
    # the pool's default stage kernel for the class
    f.set_tuning(G.TUNE_STAGE_VARIANT, 0 if (w.dim == 3 and w.degree == 3) else 1)
    u = f.project_ic(w.ic_kind, w.ic_params)
    work, dt = f.new_work(), torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(w.steps):
        f.step(u, work, dt, w.cfl)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def test_served_results_equal_solo_solves():
    from paper_2502_12620_amd.serve import Request, Server

    reqs = [Request(i, t, w) for i, (t, w) in enumerate(_requests())]
    classes = sorted({(r.workload.dim, r.workload.degree, r.workload.n_cell) for r in reqs})
    # one budget for all classes, twice the largest request's footprint:
    # requests queue for room, pools grow, shrink and move their members
    from paper_2502_12620_amd.serve import slot_bytes

    foot = [slot_bytes(r.workload.dim, r.workload.degree, r.workload.n_cell) * int(np.prod(r.workload.roots))
            for r in reqs]
    srv = Server(classes, hbm_budget=2 * max(foot), max_members=2, keep_results=True)
    done = srv.run(reqs)
    assert len(done) == len(reqs)
    assert srv.full_waits > 0, "no request had to wait for room"
    assert srv.moved > 0, "no pool was resized with members in it"
    assert srv.peak_bytes <= 2 * max(foot)
    for r in done:
        assert r.done >= r.admitted >= r.arrival
        got = r.result.cpu().numpy()
        assert np.array_equal(got, _alone(r.workload)), f"request {r.rid} differs from its solo solve"


def test_served_stream_sample_matches_the_oracle():
    """A sample of the served stream (seed 12620, 200 requests/s): its first
    four 2-D requests of at most 32 root blocks and 150 steps (degrees 1, 2,
    3, 3), served together by the request loop at their arrival times,
    against the FP64 oracle: relative L2 of the density and of all
    coefficients within 1e-12, the bar of the FP64 parity tests."""
    import oracle as O
    from paper_2502_12620_amd.serve import Request, Server

    stream = W.served_requests(1000, seed=12620, rate=200.0)
    pick = [(t, w) for t, w in stream if w.dim == 2 and np.prod(w.roots) <= 32 and w.steps <= 150][:4]
    t0 = pick[0][0]
    reqs = [Request(i, t - t0, w) for i, (t, w) in enumerate(pick)]
    classes = sorted({(r.workload.dim, r.workload.degree, r.workload.n_cell) for r in reqs})
    srv = Server(classes, hbm_budget=4e9, keep_results=True)
    done = srv.run(reqs)
    for r in sorted(done, key=lambda r: r.rid):
        w = r.workload
        f = O.Forest(w.dim, w.degree, w.n_cell, w.roots, w.lo, w.hi, w.bc, w.max_level, w.gamma)
        u = f.project_ic(w.ic_kind, w.ic_params)
        for _ in range(w.steps):
            f.step(u, w.cfl)
        got = r.result.cpu().numpy()
        l2_rho = np.linalg.norm(got[:, 0] - u[:, 0]) / np.linalg.norm(u[:, 0])
        l2_all = np.linalg.norm(got - u) / np.linalg.norm(u)
        print(f"served request p={w.degree} roots={w.roots} steps={w.steps}: L2 density {l2_rho:.2e}, all {l2_all:.2e}")
        assert l2_rho <= 1e-12 and l2_all <= 1e-12
