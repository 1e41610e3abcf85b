"""GPU tests of the serving pool (lfsr_pool_*): every job's result equals
its solo lfsr_solve bit for bit (the pool runs the same kernels on the same
resident state, replayed from a captured graph each tick), admission follows
the arena budget, and input errors come back per job."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from helpers import CASES, disp_bound, make_case  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lfsr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_05047_amd import lfsr as mod
    mod.load()
    return mod


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


def _jobs(lfsr):
    """Mixed angular sizes, spatial sizes, scales and storage types."""
    out = []
    for name, over in [("c1", {}), ("ragged", {}), ("single", {}), ("c1", {"storage": "f16", "n_iter": 7}),
                       ("ragged", {"storage": "bf16", "n_iter": 9})]:
        c = make_case(CASES[name])
        prm = lfsr.make_params(c["cfg"], disp_bound=disp_bound(c["cfg"]), **over)
        out.append((prm, _t(c["y"]), _t(c["disp"])))
    return out


def _solo(lfsr, prm, y, d):
    x, _ = lfsr.Solver(prm).lfsr_solve(y, d, stats=False)
    torch.cuda.synchronize()
    return x.cpu().numpy()


def _drain(pool, done, max_ticks=1000):
    for _ in range(max_ticks):
        for jid, out, st, it in pool.lfsr_pool_poll():
            torch.cuda.synchronize()
            done[jid] = (out.cpu().numpy(), st, it)
        if pool.lfsr_pool_info()["active"] == 0 and pool.lfsr_pool_info()["retiring"] == 0:
            return
        pool.lfsr_pool_tick()
        torch.cuda.synchronize()
    raise AssertionError("pool did not drain")


def test_pool_results_equal_solo_solves(lfsr):
    jobs = _jobs(lfsr)
    solo = [_solo(lfsr, *j) for j in jobs]
    need = sum(lfsr.workspace_bytes(j[0]) + 256 for j in jobs)
    pool = lfsr.Pool(need, max_slots=8)
    ids = [pool.lfsr_pool_submit(*j) for j in jobs]
    assert all(i is not None for i in ids)
    done = {}
    _drain(pool, done)
    for i, (jid, ref) in enumerate(zip(ids, solo)):
        x, st, it = done[jid]
        assert st == lfsr.LFSR_OK and it == jobs[i][0].admm_iters
        np.testing.assert_array_equal(x, ref)
    pool.close()


def test_pool_staggered_arrivals_and_budget(lfsr):
    """Arena for two c1-sized jobs: a third waits (EBUSY) until one is
    harvested; jobs admitted mid-stream still match their solo results."""
    jobs = _jobs(lfsr)
    c1 = jobs[0]
    big = lfsr.workspace_bytes(c1[0])
    pool = lfsr.Pool(2 * big + 512, max_slots=4)
    solo = _solo(lfsr, *c1)
    a = pool.lfsr_pool_submit(*c1)
    for _ in range(3):
        pool.lfsr_pool_tick()
    b = pool.lfsr_pool_submit(*c1)
    assert a is not None and b is not None
    assert pool.lfsr_pool_submit(*c1) is None  # no room now
    with pytest.raises(lfsr.LfsrError):  # never fits
        huge = lfsr.make_params(dict(CASES["c1"], sy=2048, sx=2048), disp_bound=2.0)
        pool.lfsr_pool_submit(huge, c1[1], c1[2])
    done, waiting, c = {}, True, None
    for _ in range(200):
        for jid, out, st, it in pool.lfsr_pool_poll():
            torch.cuda.synchronize()
            done[jid] = out.cpu().numpy()
        if waiting:
            c = pool.lfsr_pool_submit(*c1)
            waiting = c is None
        info = pool.lfsr_pool_info()
        if not waiting and info["active"] == 0 and info["retiring"] == 0:
            break
        pool.lfsr_pool_tick()
        torch.cuda.synchronize()  # one tick at a time: the host must not run ahead of the device
    assert c is not None and set(done) == {a, b, c}
    for jid in (a, b, c):
        np.testing.assert_array_equal(done[jid], solo)
    assert pool.lfsr_pool_info()["free"] >= 2 * big
    pool.close()


def test_pool_reports_input_errors_per_job(lfsr):
    jobs = _jobs(lfsr)
    prm, y, d = jobs[0]
    bad = y.clone()
    bad[0, 0, 0] = float("nan")
    pool = lfsr.Pool(3 * lfsr.workspace_bytes(prm), max_slots=4)
    good_id = pool.lfsr_pool_submit(prm, y, d)
    bad_id = pool.lfsr_pool_submit(prm, bad, d)
    done = {}
    _drain(pool, done)
    assert done[good_id][1] == lfsr.LFSR_OK
    assert done[bad_id][1] == lfsr.LFSR_ENONFINITE
    pool.close()


def test_pool_unsynchronised_ticks_with_admissions(lfsr):
    """A serving loop does not wait for each tick: jobs admitted while earlier
    graph launches are still executing force a new graph each time, and the
    replaced graphs must outlive their launches.  Results stay bit-identical."""
    jobs = _jobs(lfsr)
    solo = [_solo(lfsr, *j) for j in jobs[:3]]
    pool = lfsr.Pool(sum(lfsr.workspace_bytes(j[0]) + 256 for j in jobs[:3]), max_slots=8)
    ids = [pool.lfsr_pool_submit(*jobs[0])]
    for _ in range(3):
        pool.lfsr_pool_tick()
    ids.append(pool.lfsr_pool_submit(*jobs[1]))
    for _ in range(2):
        pool.lfsr_pool_tick()
    ids.append(pool.lfsr_pool_submit(*jobs[2]))
    done = {}
    for _ in range(1000):
        for jid, out, st, it in pool.lfsr_pool_poll():
            torch.cuda.synchronize()
            done[jid] = out.cpu().numpy()
        info = pool.lfsr_pool_info()
        if info["active"] == 0:
            if info["retiring"] == 0:
                break
            torch.cuda.synchronize()
        pool.lfsr_pool_tick()
    assert set(done) == set(ids)
    for jid, ref in zip(ids, solo):
        np.testing.assert_array_equal(done[jid], ref)
    pool.close()
