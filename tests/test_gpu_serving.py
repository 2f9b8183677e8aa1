"""Request server (bddc_server_*): continuous admission by footprint, work of
concurrent requests overlapping on the device, results independent of the
mix.

Tolerance: 0.  Every kernel is deterministic and no reduction crosses
requests, so each request's solution must have the same bits whether it runs
alone or among others, and the same bits as a direct context solve.
"""
import numpy as np
import pytest

import meshgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0910_5863_amd import BDDC, Server
    return BDDC, Server


def _requests():
    """Eight small requests in the serving recipe: Poisson and elasticity,
    8^3-16^3 elements, 2^3 substructures, layered contrast, half of them
    with adaptive face constraints."""
    specs = [
        (meshgen.POISSON, 8, 1e0, 0.0), (meshgen.ELASTICITY, 8, 1e3, 10.0),
        (meshgen.POISSON, 12, 1e4, 0.0), (meshgen.ELASTICITY, 12, 1e2, 10.0),
        (meshgen.POISSON, 16, 1e2, 2.0), (meshgen.ELASTICITY, 8, 1e5, 0.0),
        (meshgen.ELASTICITY, 12, 1e0, 10.0), (meshgen.POISSON, 12, 1e6, 10.0),
    ]
    out = []
    for i, (kind, n, contrast, tau) in enumerate(specs):
        req = dict(id=i, kind=kind, n=n, s=2, contrast=contrast, seed=1000 + i)
        out.append((meshgen.request_problem(req), tau))
    return out


def test_server_results_alone_and_in_the_mix():
    BDDC, Server = _gpu()
    reqs = _requests()
    # alone: one request in flight at a time, each waited for before the next
    alone = []
    srv = Server(max_active=1)
    for p, tau in reqs:
        rid = srv.submit(p, tau)
        u, info = srv.wait(rid)
        assert info.state == 2, info.error
        alone.append((u, info))
    srv.close()
    # in the mix: all submitted at once, four workers, a budget that fits
    # about three of the largest footprints at a time
    fps = sorted(info.footprint_bytes for _, info in alone)
    budget = 3.0 * fps[-1]
    srv = Server(max_active=4, hbm_budget_bytes=budget)
    ids = [srv.submit(p, tau) for p, tau in reqs]
    mix = [srv.wait(i) for i in ids]
    srv.close()
    for (ua, ia), (um, im) in zip(alone, mix):
        assert im.state == 2, im.error
        assert ia.pcg.converged and im.pcg.converged
        assert ia.pcg.iters == im.pcg.iters
        assert np.array_equal(ua, um)
        assert ia.nc == im.nc and ia.omega == im.omega
    # admission: whenever a request started, the requests then in flight
    # (itself included) fit in the budget, unless it ran alone
    for i, (_, im) in enumerate(mix):
        live = [m for _, m in mix if m.start_s <= im.start_s < m.done_s]
        if len(live) > 1:
            assert sum(m.footprint_bytes for m in live) <= budget * (1 + 1e-12)
    # overlap: some requests were in flight together
    assert any(sum(1 for _, m in mix if m.start_s <= im.start_s < m.done_s) > 1 for _, im in mix)
    # the same bits as a direct context solve
    p, tau = reqs[3]
    b = BDDC()
    b.setup(p, "ce")
    if tau > 0:
        b.adapt(tau)
    b.factor()
    u, _ = b.pcg_solve(torch.from_numpy(p.f))
    assert np.array_equal(u.cpu().numpy()[:, 0], alone[3][0])
    b.close()


def test_server_solution_solves_the_assembled_system():
    _, Server = _gpu()
    from oracle.fem import Substructures
    p, tau = _requests()[1]
    srv = Server(max_active=2)
    u, info = srv.wait(srv.submit(p, tau))
    srv.close()
    assert info.state == 2, info.error
    K = Substructures(p).assembled()
    r = np.linalg.norm(p.f - K @ u) / np.linalg.norm(p.f)
    assert r < 1e-7, r


def test_server_reports_request_errors():
    """A load of the wrong length fails that request only (BDDC_ERR_ARG in
    its record); the next request is served normally."""
    _, Server = _gpu()
    from paper_0910_5863_amd import binding
    p, _ = _requests()[0]
    srv = Server(max_active=1)
    mesh, part, cons, _arrays = binding._marshal(p, "ce")
    f = np.ones(p.f.shape[0] + 1)
    rid = binding.bddc_server_submit(srv.h, mesh, part, cons, 0.0, f, binding.bddc_pcg_params(0, 0))
    srv._n[rid] = f.shape[0]
    u, info = srv.wait(rid)
    assert info.state == 3 and info.status == 1
    ok = srv.submit(p)
    u, info = srv.wait(ok)
    assert info.state == 2
    srv.close()


def test_server_resident_factors():
    """resident_bytes > 0: requests on one problem with different loads are
    served by one factored context.  Each solution has the bits of a fresh
    solve of its load; every request after the first reports reuse; a
    different problem in between is served normally; with a limit below one
    footprint the idle context is destroyed and the next request on the
    problem factors it again; under a budget that holds one of two problems,
    each evicts the other's idle context."""
    _, Server = _gpu()
    p, tau = _requests()[3]
    rng = np.random.default_rng(7)
    loads = [p.f] + [p.f * rng.uniform(0.5, 2.0, p.f.shape) for _ in range(5)]
    other, tau_o = _requests()[0]
    fresh = []
    srv = Server(max_active=1)
    for f in loads:
        u, info = srv.wait(srv.submit(p, tau, f=f))
        assert info.state == 2 and info.reused == 0, info.error
        fresh.append((u, info))
    u_o, i_o = srv.wait(srv.submit(other, tau_o))
    srv.close()
    srv = Server(max_active=2, resident_bytes=1e12)
    first = srv.wait(srv.submit(p, tau, f=loads[0]))
    ids = [srv.submit(p, tau, f=f) for f in loads[1:3]]
    ids.append(srv.submit(other, tau_o))
    ids += [srv.submit(p, tau, f=f) for f in loads[3:]]
    got = [first] + [srv.wait(i) for i in ids]
    srv.close()
    u_mid, i_mid = got.pop(3)
    assert i_mid.state == 2 and np.array_equal(u_mid, u_o) and i_mid.reused == 0
    assert got[0][1].reused == 0
    for k, ((u, info), (uf, inf_f)) in enumerate(zip(got, fresh)):
        assert info.state == 2, info.error
        assert k == 0 or info.reused == 1
        assert np.array_equal(u, uf)
        assert info.pcg.iters == inf_f.pcg.iters
        assert info.nc == inf_f.nc and info.omega == inf_f.omega
    # a limit below one footprint: nothing stays resident
    srv = Server(max_active=1, resident_bytes=1.0)
    a = srv.wait(srv.submit(p, tau, f=loads[1]))
    b = srv.wait(srv.submit(p, tau, f=loads[2]))
    srv.close()
    assert a[1].reused == 0 and b[1].reused == 0
    assert np.array_equal(a[0], fresh[1][0]) and np.array_equal(b[0], fresh[2][0])
    # a budget below the two problems' footprints: each new problem evicts
    # the idle context of the other, and a problem that stays resident is
    # reused
    budget = fresh[0][1].footprint_bytes + i_o.footprint_bytes - 1.0
    srv = Server(max_active=1, resident_bytes=1e12, hbm_budget_bytes=budget)
    seq = [(p, tau, loads[1]), (other, tau_o, None), (p, tau, loads[2]), (p, tau, loads[3])]
    res = [srv.wait(srv.submit(q, t, f=f)) for q, t, f in seq]
    srv.close()
    assert [r[1].state for r in res] == [2, 2, 2, 2]
    assert [r[1].reused for r in res] == [0, 0, 0, 1]
    assert np.array_equal(res[1][0], u_o)
    for (u, _), k in zip([res[0], res[2], res[3]], (1, 2, 3)):
        assert np.array_equal(u, fresh[k][0])


def test_server_blocks_on_a_resident_problem_match_the_oracle():
    """Requests queued on one resident problem are solved as block PCGs (up
    to 8 loads each): every served solution matches the oracle's solution of
    its load to 1e-8 (element-wise, relative to the largest entry) and has
    the bits of a direct single solve."""
    BDDC, Server = _gpu()
    from oracle.solver import OracleBDDC
    p, tau = _requests()[5]  # elasticity 8^3, contrast 1e5, c+e constraints
    assert tau == 0.0
    rng = np.random.default_rng(11)
    loads = [p.f] + [p.f * rng.uniform(0.5, 2.0, p.f.shape) + rng.standard_normal(p.f.shape)
                     for _ in range(12)]
    srv = Server(max_active=1, resident_bytes=1e12)
    ids = [srv.submit(p, tau, f=f) for f in loads]
    got = [srv.wait(i) for i in ids]
    srv.close()
    o = OracleBDDC(p, "ce")
    b = BDDC()
    b.setup(p, "ce")
    b.factor()
    for k, ((u, info), f) in enumerate(zip(got, loads)):
        assert info.state == 2, info.error
        assert k == 0 or info.reused == 1
        ref = o.solve(f)["u"]
        err = float(np.abs(u - ref).max() / np.abs(ref).max())
        assert err < 1e-8, (k, err)
        u1, _ = b.pcg_solve(torch.from_numpy(f))
        assert np.array_equal(u, u1.cpu().numpy()[:, 0]), k
    b.close()
    batches = [info.batch for _, info in got]
    assert max(batches) > 1 and max(batches) <= 8, batches
