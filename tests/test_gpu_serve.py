"""The solve server (continuous batching) through the C ABI: every served solve equals the same
solve run alone (bitwise: support, beta, iteration count, status, loss trace), whatever else was
admitted, queued or retired around it; FP64 served solves also match the oracle at the fit bars.
Admission respects the slot count and the device-memory budget; bad requests are rejected.
"""
import numpy as np
import pytest

from oracle import oracle
from paper_1608_01398_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1608_01398_amd import iht  # noqa: E402


def say(*a):
    print(*a, flush=True)


def dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


@pytest.fixture(scope="module")
def prob():
    p = synth.make_problem("c1", seed=31, n=1200, p=6000)
    traits = [synth.make_trait(p["bed"], p["n"], p["q"], 10, (0.2, 0.5), seed=300 + e)[0] for e in range(16)]
    p["traits"] = np.stack(traits)
    p["geno"] = iht.Geno(p["bed"], p["n"])
    return p


def requests(prob):
    """(subset, trait rows, ks) of a mixed stream: different subsets, trait counts and sizes."""
    n = prob["n"]
    rng = np.random.default_rng(5)
    subs = [synth.make_subset(n, 900, 1), None, synth.make_subset(n, 1000, 2), synth.make_subset(n, 700, 3),
            synth.make_subset(n, 1100, 4)]
    sizes = [5, 1, 7, 12, 2]
    out = []
    for s, T in zip(subs, sizes):
        rows = rng.choice(len(prob["traits"]), T, replace=False)
        ks = rng.integers(2, 17, T)
        out.append((s, rows, ks))
    return out


def alone(prob, subset, row, k, precision, Z=None):
    g = prob["geno"]
    return iht.fit(g, iht.Stats(g, subset), dev(prob["traits"][row]), int(k), precision=precision,
                   Z=None if Z is None else dev(Z, torch.float32))


def assert_same(res, j, ref):
    k = int(res["ks"][j])
    it = int(res["n_iter"][j])
    assert int(res["statuses"][j]) == ref["status"]
    assert it == ref["n_iter"]
    assert torch.equal(res["support"][j, :k], ref["support"])
    assert torch.all(res["support"][j, k:] == -1)
    assert torch.equal(res["beta_S"][j, :k], ref["beta_S"])
    assert torch.equal(res["beta_cov"][j], ref["beta_cov"])
    assert torch.equal(res["loss_trace"][j, :it + 1], ref["loss_trace"])


@pytest.mark.parametrize("precision", [iht.FP64, iht.FP32, iht.MIXED_I8])
def test_served_equals_alone_with_staggered_arrivals(prob, precision):
    """Requests arrive between steps while others iterate; one waits for slots; all equal alone."""
    say(f"serve staggered precision={precision}")
    srv = iht.Server(prob["geno"], slots=16, kmax=16, hbm_budget=8 << 30, precision=precision)
    reqs = requests(prob)
    ids = []
    Ys = [dev(prob["traits"][rows]) for _, rows, _ in reqs]
    ids.append(srv.submit(Ys[0], reqs[0][2], reqs[0][0]))
    ids.append(srv.submit(Ys[1], reqs[1][2], reqs[1][0]))
    srv.step()
    srv.step()
    ids.append(srv.submit(Ys[2], reqs[2][2], reqs[2][0]))
    srv.step()
    ids.append(srv.submit(Ys[3], reqs[3][2], reqs[3][0]))  # 12 traits: waits for free slots
    ids.append(srv.submit(Ys[4], reqs[4][2], reqs[4][0]))  # queued behind it (arrival order)
    inf = srv.info()
    assert inf["slots_busy"] <= 16
    peak_busy = 0
    for _ in range(2000):
        inf = srv.info()
        peak_busy = max(peak_busy, inf["slots_busy"])
        if inf["queued"] == 0 and inf["running"] == 0:
            break
        srv.step()
    assert inf["completed"] == 5 and peak_busy <= 16
    for rid, (subset, rows, ks) in zip(ids, reqs):
        res = srv.result(rid)
        for j, (row, k) in enumerate(zip(rows, ks)):
            assert_same(res, j, alone(prob, subset, row, k, precision))
    srv.close()


def test_served_fp64_matches_oracle(prob):
    srv = iht.Server(prob["geno"], slots=8, kmax=16, hbm_budget=8 << 30)
    subset, rows, ks = requests(prob)[2]
    rid = srv.submit(dev(prob["traits"][rows]), ks, subset)
    srv.run_until_idle()
    res = srv.result(rid)
    for j, (row, k) in enumerate(zip(rows, ks)):
        ref = oracle.fit(prob["bed"], prob["n"], prob["traits"][row], int(k), intercept=True, subset=subset)
        assert int(res["statuses"][j]) == ref["status"]
        assert np.array_equal(res["support"][j, :k].cpu().numpy(), ref["support"])
        scale = np.abs(ref["beta_S"]).max()
        assert np.abs(res["beta_S"][j, :k].cpu().numpy() - ref["beta_S"]).max() <= 1e-6 * scale
        assert int(res["n_iter"][j]) == ref["n_iter"]
        np.testing.assert_allclose(res["loss_trace"][j, :ref["n_iter"] + 1].cpu().numpy(), ref["loss_trace"],
                                   rtol=1e-9)
    srv.close()


def test_served_mixed_matches_fp64_and_oracle_above_effects(prob):
    """The serving workload's regime on a small matrix: int8 matrix-core served solves with k above
    the traits' 10 effects (k up to 40, near-ties among noise SNPs), two requests on different subject
    sets sharing the slots. Each equals the FP64 fit of the same solve (status, support, iteration
    count; beta within 1e-6, loss trace within 1e-9 relative), and two of them equal the oracle."""
    srv = iht.Server(prob["geno"], slots=16, kmax=40, hbm_budget=8 << 30, precision=iht.MIXED_I8)
    reqs = [(synth.make_subset(prob["n"], 1000, 9), np.array([0, 3, 5, 8, 11, 14]), np.array([12, 20, 25, 30, 35, 40])),
            (None, np.array([1, 2, 6, 7]), np.array([40, 33, 18, 27]))]
    ids = [srv.submit(dev(prob["traits"][rows]), ks, subset) for subset, rows, ks in reqs]
    srv.run_until_idle()
    checked = 0
    for rid, (subset, rows, ks) in zip(ids, reqs):
        res = srv.result(rid)
        for j, (row, k) in enumerate(zip(rows, ks)):
            k = int(k)
            ref = alone(prob, subset, row, k, iht.FP64)
            it = int(ref["n_iter"])
            assert int(res["statuses"][j]) == ref["status"], (rid, j)
            assert int(res["n_iter"][j]) == it, (rid, j)
            assert torch.equal(res["support"][j, :k], ref["support"]), (rid, j)
            b64 = ref["beta_S"].cpu().numpy()
            assert np.abs(res["beta_S"][j, :k].cpu().numpy() - b64).max() <= 1e-6 * np.abs(b64).max()
            np.testing.assert_allclose(res["loss_trace"][j, :it + 1].cpu().numpy(),
                                       ref["loss_trace"].cpu().numpy(), rtol=1e-9)
            if j == 0:
                o = oracle.fit(prob["bed"], prob["n"], prob["traits"][row], k, intercept=True, subset=subset)
                assert int(res["n_iter"][j]) == o["n_iter"]
                assert np.array_equal(res["support"][j, :k].cpu().numpy(), o["support"])
                checked += 1
    assert checked == 2
    srv.close()


def test_budget_limits_admission_to_one_subject_set(prob):
    """A budget with room for one statistics block admits one request at a time."""
    g = prob["geno"]
    big = iht.Server(g, slots=16, kmax=16, hbm_budget=8 << 30)
    inf = big.info()
    big.close()
    n, p = prob["n"], prob["p"]
    n_pad = (n + 31) // 32 * 32
    block = ((2 * p + n_pad) * 8 + (n_pad // 32) * 4 + 255) // 256 * 256
    slot_bytes = inf["device_bytes"] - inf["stats_blocks"] * block
    srv = iht.Server(g, slots=16, kmax=16, hbm_budget=slot_bytes + block + block // 2)
    assert srv.info()["stats_blocks"] == 1
    reqs = requests(prob)[:3]
    ids = [srv.submit(dev(prob["traits"][rows]), ks, s) for s, rows, ks in reqs]
    for _ in range(2000):
        inf = srv.info()
        assert inf["running"] <= 1
        if inf["queued"] == 0 and inf["running"] == 0:
            break
        srv.step()
    for rid, (subset, rows, ks) in zip(ids, reqs):
        res = srv.result(rid)
        for j, (row, k) in enumerate(zip(rows, ks)):
            assert_same(res, j, alone(prob, subset, row, k, iht.FP64))
    with pytest.raises(iht.IHTError) as e:
        iht.Server(g, slots=16, kmax=16, hbm_budget=slot_bytes)
    assert e.value.code == iht.ENOMEM
    srv.close()


def test_served_covariates_and_nonfinite_trait(prob):
    g = prob["geno"]
    n = prob["n"]
    Z = synth.make_covariates(n, 2, 9)
    srv = iht.Server(g, slots=6, kmax=12, hbm_budget=8 << 30, Z=dev(Z, torch.float32))
    Y = prob["traits"][[0, 1, 2]].copy()
    subset = synth.make_subset(n, 1000, 7)
    inside = int(np.flatnonzero(subset)[3])
    Y[1, inside] = np.nan
    ks = np.array([4, 6, 9])
    rid = srv.submit(dev(Y), ks, subset)
    srv.run_until_idle()
    res = srv.result(rid)
    assert int(res["statuses"][1]) == iht.ENONFINITE
    assert torch.all(res["support"][1] == -1)
    for j in (0, 2):
        ref = iht.fit(g, iht.Stats(g, subset), dev(Y[j]), int(ks[j]), Z=dev(Z, torch.float32))
        assert_same(res, j, ref)
    srv.close()


def test_server_rejects_bad_requests(prob):
    g = prob["geno"]
    n = prob["n"]
    srv = iht.Server(g, slots=4, kmax=8, hbm_budget=8 << 30)
    Y = dev(prob["traits"][:5])
    for Yb, ks, sub in ((Y, [3] * 5, None),                         # more traits than slots
                        (Y[:2], [3, 9], None),                      # k > kmax
                        (Y[:1], [3], np.full(n, 2, np.uint8)),      # subset entries not 0/1
                        (Y[:1], [3], np.zeros(n, np.uint8))):       # empty subject set
        with pytest.raises(iht.IHTError) as e:
            srv.submit(Yb, ks, sub)
        assert e.value.code == iht.EINVAL
    with pytest.raises(iht.IHTError) as e:
        srv.done(99)
    assert e.value.code == iht.EINVAL
    assert srv.info()["queued"] == 0
    srv.close()


def test_server_idle_steps_and_info(prob):
    """Steps with nothing queued do nothing; the counters follow a request through the server."""
    srv = iht.Server(prob["geno"], slots=8, kmax=10, hbm_budget=8 << 30)
    assert srv.step() == 0
    inf = srv.info()
    assert (inf["queued"], inf["running"], inf["completed"], inf["slots_busy"], inf["turns"]) == (0, 0, 0, 0, 0)
    assert inf["slots"] == 8 and inf["stats_blocks"] == 8 and inf["device_bytes"] > 0
    rid = srv.submit(dev(prob["traits"][:3]), [4, 6, 8])
    assert srv.info()["queued"] == 1 and not srv.done(rid)
    srv.step()
    inf = srv.info()
    assert inf["queued"] == 0 and inf["slots_busy"] + 3 * inf["completed"] == 3
    srv.run_until_idle()
    inf = srv.info()
    assert inf["completed"] == 1 and inf["slots_busy"] == 0 and inf["turns"] >= 1 and srv.done(rid)
    res = srv.result(rid)
    assert list(res["statuses"]) == [iht.OK] * 3
    srv.close()
