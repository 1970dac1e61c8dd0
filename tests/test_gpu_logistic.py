"""Logistic IHT (the extension the Discussion names) through the C ABI against the FP64 oracle:
identical supports, status and iteration counts, beta within 1e-6 relative, loss traces within 1e-9
relative; a logistic solve is the same alone, in a batch and served; unsupported combinations are
rejected.
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
    n, p = 1500, 8000
    bed, q = synth.make_genotypes(n, p, 61)
    ys = [synth.make_binary_trait(bed, n, q, 8, (0.3, 0.8), seed=610 + e)[0] for e in range(6)]
    return dict(bed=bed, n=n, p=p, q=q, ys=np.stack(ys), geno=iht.Geno(bed, n))


def check(got, ref):
    assert got["status"] == ref["status"], (got["status"], ref["status"])
    sup = got["support"].cpu().numpy()
    assert np.array_equal(sup, ref["support"]), (sup, ref["support"])
    scale = np.abs(ref["beta_S"]).max()
    assert np.abs(got["beta_S"].cpu().numpy() - ref["beta_S"]).max() <= 1e-6 * scale
    if len(ref["beta_cov"]):
        np.testing.assert_allclose(got["beta_cov"].cpu().numpy(), ref["beta_cov"], rtol=1e-6, atol=1e-6 * scale)
    assert got["n_iter"] == ref["n_iter"], (got["n_iter"], ref["n_iter"])
    np.testing.assert_allclose(got["loss_trace"].cpu().numpy(), ref["loss_trace"], rtol=1e-9)


@pytest.mark.parametrize("t,k", [(0, 8), (1, 3), (2, 15)])
def test_logistic_fit_matches_oracle(prob, t, k):
    say(f"logistic fit trait {t} k={k}")
    g = prob["geno"]
    got = iht.fit(g, iht.Stats(g), dev(prob["ys"][t]), k, family=iht.LOGISTIC)
    ref = oracle.fit(prob["bed"], prob["n"], prob["ys"][t], k, family=1)
    check(got, ref)
    tr = ref["loss_trace"]
    assert np.all(np.diff(tr) <= 1e-12 * tr[0])


def test_logistic_covariates_and_subset(prob):
    g = prob["geno"]
    n = prob["n"]
    Z = synth.make_covariates(n, 2, 62)
    m = synth.make_subset(n, 1100, 6)
    got = iht.fit(g, iht.Stats(g, m), dev(prob["ys"][3]), 6, Z=dev(Z, torch.float32), family=iht.LOGISTIC)
    ref = oracle.fit(prob["bed"], n, prob["ys"][3], 6, Z=Z, subset=m, family=1)
    check(got, ref)


def test_logistic_batched_and_served_equal_alone(prob):
    g = prob["geno"]
    s = iht.Stats(g)
    ks = [4, 8, 12, 8]
    Y = prob["ys"][[0, 1, 4, 5]]
    bat = iht.fit_batch(g, [s] * 4, dev(Y), ks, family=iht.LOGISTIC)
    srv = iht.Server(g, slots=4, kmax=12, hbm_budget=4 << 30, family=iht.LOGISTIC)
    rid = srv.submit(dev(Y), ks)
    srv.run_until_idle()
    sv = srv.result(rid)
    srv.close()
    for j, k in enumerate(ks):
        alone = iht.fit(g, s, dev(Y[j]), k, family=iht.LOGISTIC)
        it = alone["n_iter"]
        for res in (bat, sv):
            assert int(res["n_iter"][j]) == it
            assert torch.equal(res["support"][j, :k], alone["support"])
            assert torch.equal(res["beta_S"][j, :k], alone["beta_S"])
            assert torch.equal(res["loss_trace"][j, :it + 1], alone["loss_trace"])


def test_logistic_rejections(prob):
    g = prob["geno"]
    s = iht.Stats(g)
    y = dev(prob["ys"][0])
    for prec in (iht.FP32, iht.MIXED_I8):
        with pytest.raises(iht.IHTError) as e:
            iht.fit(g, s, y, 5, family=iht.LOGISTIC, precision=prec)
        assert e.value.code == iht.EUNSUPPORTED
    with pytest.raises(iht.IHTError) as e:
        iht.cv(g, y, [2, 4], synth.make_folds(prob["n"], 3, 1), 3, family=iht.LOGISTIC)
    assert e.value.code == iht.EUNSUPPORTED
    y2 = prob["ys"][0].copy()
    y2[10] = 1.5
    with pytest.raises(iht.IHTError) as e:
        iht.fit(g, s, dev(y2), 5, family=iht.LOGISTIC)
    assert e.value.code == iht.ENONFINITE
    with pytest.raises(iht.IHTError) as e:
        iht.fit(g, s, y, 5, family=7)
    assert e.value.code == iht.EINVAL
