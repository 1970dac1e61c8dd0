"""Parity at the full workload sizes, in the launch configurations the benchmark times.

The oracle checks outputs it can compute one by one: gradient entries of sampled SNPs (every SNP's
statistics and gradient entry depend on its own row only, so the oracle runs on the sampled rows),
and whole fits where an oracle fit finishes in seconds (n = 5000, p = 500,000). At n = 20,000,
p = 2,000,000 (10 GB packed) an oracle fit takes many minutes, so two oracle solves are stored as
goldens (tests/golden/make_c5_goldens.py) and the other fits are checked by properties that hold
at any size: a converged fit is the least-squares fit of y on its support and the unpenalised
columns (the fixed point of the IHT map on a fixed support), and the int8 matrix-core solves take
the FP64 solves' decisions (same statuses, supports and iteration counts).
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


def sampled_gradient_ref(bed, n, cols, r, subset=None):
    sub = np.ascontiguousarray(bed[cols])
    u, v = oracle.stats(sub, n, subset)
    return oracle.gradient(sub, n, u, v, r, subset)


def ls_fit(bed, n, y, support, Z=None, intercept=True, subset=None):
    """Least squares of y on the standardised support columns and the unpenalised columns."""
    sub = np.ascontiguousarray(bed[np.asarray(support)])
    u, v = oracle.stats(sub, n, subset)
    X = oracle.standardize(sub, n, u, v).T  # [n, k]
    cols = [X]
    if Z is not None:
        cols.append(np.asarray(Z, dtype=np.float64).T)
    if intercept:
        cols.append(np.ones((n, 1)))
    A = np.concatenate(cols, axis=1)
    rows = slice(None) if subset is None else subset.astype(bool)
    coef, *_ = np.linalg.lstsq(A[rows], y[rows], rcond=None)
    k = len(support)
    return coef[:k], coef[k:]


# ------------------------------------------------------------------ n = 5000, p = 500,000

@pytest.fixture(scope="module")
def c2():
    prob = synth.make_problem("c2", 1)
    prob["geno"] = iht.Geno(prob["bed"], prob["n"])
    prob["cols"] = np.sort(np.random.default_rng(0).choice(prob["p"], 3000, replace=False))
    return prob


@pytest.mark.parametrize("precision,bar", [(iht.FP64, 1e-12), (iht.FP32, 2e-6)])
def test_c2_gradient_sampled(c2, precision, bar):
    say(f"c2 gradient precision={precision}")
    g = iht.gradient(c2["geno"], iht.Stats(c2["geno"]), dev(c2["y"]), precision).cpu().numpy()
    ref = sampled_gradient_ref(c2["bed"], c2["n"], c2["cols"], c2["y"])
    got = g[c2["cols"]]
    assert np.linalg.norm(got - ref) <= bar * np.linalg.norm(ref)
    if precision == iht.FP64:
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_c2_fit_matches_oracle(c2):
    say("c2 fit vs oracle (one oracle solve, ~10 s)")
    res = iht.fit(c2["geno"], iht.Stats(c2["geno"]), dev(c2["y"]), c2["k"])
    ref = oracle.fit(c2["bed"], c2["n"], c2["y"], c2["k"], intercept=True)
    assert res["status"] == ref["status"] == iht.OK
    assert np.array_equal(res["support"].cpu().numpy(), ref["support"])
    assert np.abs(res["beta_S"].cpu().numpy() - ref["beta_S"]).max() <= 1e-6 * np.abs(ref["beta_S"]).max()
    assert res["n_iter"] == ref["n_iter"]
    np.testing.assert_allclose(res["loss_trace"].cpu().numpy(), ref["loss_trace"], rtol=1e-9)


def test_c3_batched_pass_sampled(c2):
    """The 108-solve layout (5 training folds x k = 1..20 + 8 traits on all subjects): the matrix-core
    pass on sampled SNPs of sampled solves, each with its own subject set."""
    n = c2["n"]
    fold = synth.make_folds(n, 5, 1)
    masks = [(fold != f).astype(np.uint8) for f in range(5)]
    stats = [iht.Stats(c2["geno"], m) for m in masks] + [iht.Stats(c2["geno"])]
    which = [f for f in range(5) for _ in range(20)] + [5] * 8
    R = np.random.default_rng(3).standard_normal((108, n))
    G = iht.gradient_batch(c2["geno"], [stats[w] for w in which], dev(R)).cpu().numpy()
    for t in (0, 37, 99, 104):
        m = masks[which[t]] if which[t] < 5 else None
        ref = sampled_gradient_ref(c2["bed"], n, c2["cols"], R[t], m)
        assert np.linalg.norm(G[t, c2["cols"]] - ref) <= 2e-6 * np.linalg.norm(ref), t


def test_c3_batched_fit_sample_matches_oracle(c2):
    """The 108-solve layout in one int8 matrix-core batch (5 training folds x k = 1..20 on the trait,
    plus 8 further traits at k = 20 on all subjects); 5 sampled solves against the oracle, including
    k = 1 and two of the further traits, at the FP64 bars (same status, support and iteration count,
    beta within 1e-6, loss trace within 1e-9)."""
    n = c2["n"]
    fold = synth.make_folds(n, 5, 1)
    masks = [(fold != f).astype(np.uint8) for f in range(5)]
    stats = [iht.Stats(c2["geno"], m) for m in masks] + [iht.Stats(c2["geno"])]
    ks = [k for _ in range(5) for k in range(1, 21)] + [20] * 8
    traits = [synth.make_trait(c2["bed"], n, c2["q"], 20, (0.1, 0.4), seed=100 + e)[0] for e in range(8)]
    Y = np.stack([c2["y"]] * 100 + traits)
    which = [t // 20 for t in range(100)] + [5] * 8
    res = iht.fit_batch(c2["geno"], [stats[w] for w in which], dev(Y), ks, precision=iht.MIXED_I8)
    say("c3 batched fit: statuses", np.bincount(np.asarray(res["statuses"]) + 4, minlength=7)[4:].tolist())
    for t in (0, 19, 57, 100, 107):
        k = ks[t]
        sub = masks[which[t]] if which[t] < 5 else None
        say(f"  oracle solve {t}: k={k} subset {'fold ' + str(which[t]) if sub is not None else 'all'}")
        ref = oracle.fit(c2["bed"], n, Y[t], k, intercept=True, subset=sub)
        it = int(res["n_iter"][t])
        assert int(res["statuses"][t]) == ref["status"], t
        assert it == ref["n_iter"], (t, it, ref["n_iter"])
        assert np.array_equal(res["support"][t, :k].cpu().numpy(), ref["support"]), t
        assert np.abs(res["beta_S"][t, :k].cpu().numpy() - ref["beta_S"]).max() <= 1e-6 * np.abs(ref["beta_S"]).max()
        np.testing.assert_allclose(res["loss_trace"][t, :it + 1].cpu().numpy(), ref["loss_trace"], rtol=1e-9)


# ------------------------------------------------------------------ n = 20,000, p = 2,000,000

@pytest.fixture(scope="module")
def c5():
    say("generating n=20,000 x p=2,000,000 (10 GB packed)")
    prob = synth.make_problem("c5", 2)
    prob["geno"] = iht.Geno(prob["bed"], prob["n"])
    prob["cols"] = np.sort(np.random.default_rng(1).choice(prob["p"], 1500, replace=False))
    traits = [prob["y"]]
    for e in range(31):
        y, *_ = synth.make_trait(prob["bed"], prob["n"], prob["q"], 100, (0.05, 0.3), seed=700 + e, Z=prob["Z"],
                                 intercept=1.0)
        traits.append(y)
    prob["traits"] = np.stack(traits)
    return prob


def test_c5_gradient_sampled(c5):
    g = iht.gradient(c5["geno"], iht.Stats(c5["geno"]), dev(c5["y"]), iht.FP64).cpu().numpy()
    ref = sampled_gradient_ref(c5["bed"], c5["n"], c5["cols"], c5["y"])
    got = g[c5["cols"]]
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_c5_fit_is_least_squares_on_its_support(c5):
    say("c5 FP64 fit, k = 100, 5 covariates + intercept")
    Z = dev(c5["Z"], torch.float32)
    res = iht.fit(c5["geno"], iht.Stats(c5["geno"]), dev(c5["y"]), 100, Z=Z, intercept=True)
    assert res["status"] == iht.OK
    sup = res["support"].cpu().numpy()
    assert len(np.unique(sup)) == 100 and np.all(np.diff(sup) > 0)
    b, bc = ls_fit(c5["bed"], c5["n"], c5["y"], sup, Z=c5["Z"])
    scale = np.abs(b).max()
    assert np.abs(res["beta_S"].cpu().numpy() - b).max() <= 1e-6 * scale
    np.testing.assert_allclose(res["beta_cov"].cpu().numpy(), bc, rtol=1e-6, atol=1e-6 * scale)
    # the loss trace never increases
    tr = res["loss_trace"].cpu().numpy()
    assert np.all(np.diff(tr) <= 1e-12 * tr[0])


def test_c5_batched_mixed_against_fp64(c5):
    """32 traits x k in {50, 100, 150} in one int8 matrix-core batch against the FP64 solves of the
    same traits and sizes. The matrix-core path takes the FP64 iteration's decisions (its projection
    is certified against the quantisation bound, the support's gradient is FP64), so every solve has
    the FP64 status, support and iteration count, above the number of effects (100) too, with beta
    within 1e-6 and the loss trace within 1e-9 relative."""
    Z = dev(c5["Z"], torch.float32)
    s = iht.Stats(c5["geno"])
    ks = [k for k in (50, 100, 150) for _ in range(32)]
    Y = np.concatenate([c5["traits"]] * 3)
    res = iht.fit_batch(c5["geno"], [s] * 96, dev(Y), ks, Z=Z, precision=iht.MIXED_I8)
    st = np.asarray(res["statuses"])
    say("c5 batched: statuses", np.bincount(st + 4, minlength=7)[4:].tolist(), "iterations",
        int(np.min(res["n_iter"])), "..", int(np.max(res["n_iter"])))
    ref = iht.fit_batch(c5["geno"], [s] * 96, dev(Y), ks, Z=Z, precision=iht.FP64)
    st64 = np.asarray(ref["statuses"])
    assert np.array_equal(st, st64)
    assert np.array_equal(np.asarray(res["n_iter"]), np.asarray(ref["n_iter"]))
    sup, sup64 = res["support"].cpu().numpy(), ref["support"].cpu().numpy()
    b, b64 = res["beta_S"].cpu().numpy(), ref["beta_S"].cpu().numpy()
    tr, tr64 = res["loss_trace"].cpu().numpy(), ref["loss_trace"].cpu().numpy()
    same = 0
    for t in range(96):
        k, it = ks[t], int(res["n_iter"][t])
        assert np.array_equal(sup[t, :k], sup64[t, :k]), t
        assert np.abs(b[t, :k] - b64[t, :k]).max() <= 1e-6 * np.abs(b64[t, :k]).max(), t
        np.testing.assert_allclose(tr[t, :it + 1], tr64[t, :it + 1], rtol=1e-9)
        same += 1
    say(f"identical supports and iteration counts: {same} of 96")


def test_c5_solves_match_oracle_goldens(c5):
    """Two FP64 oracle solves of this workload (k = 100 on its trait, k = 150 on a further trait of the
    same generator; 5 covariates + intercept), stored by tests/golden/make_c5_goldens.py, against the
    FP64 fit and the int8 matrix-core fit of the same problem."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_oracle_solves.json")
    doc = json.load(open(path))
    assert doc["generator"] == {"cfg": "c5", "seed": 2}
    Z = dev(c5["Z"], torch.float32)
    s = iht.Stats(c5["geno"])
    for row in doc["solves"]:
        ts, k = row["trait_seed"], row["k"]
        y = c5["traits"][0 if ts is None else 1 + (ts - 700)]
        for prec in (iht.FP64, iht.MIXED_I8):
            say(f"c5 golden: trait seed {ts} k={k} precision {prec}")
            res = iht.fit_batch(c5["geno"], [s], dev(y[None, :]), [k], Z=Z, precision=prec)
            it = int(res["n_iter"][0])
            assert int(res["statuses"][0]) == row["status"]
            assert it == row["n_iter"], (it, row["n_iter"])
            assert np.array_equal(res["support"][0, :k].cpu().numpy(), np.asarray(row["support"]))
            ref_b = np.asarray(row["beta_S"])
            assert np.abs(res["beta_S"][0, :k].cpu().numpy() - ref_b).max() <= 1e-6 * np.abs(ref_b).max()
            np.testing.assert_allclose(res["beta_cov"][0].cpu().numpy(), row["beta_cov"], rtol=1e-6,
                                       atol=1e-6 * np.abs(ref_b).max())
            np.testing.assert_allclose(res["loss_trace"][0, :it + 1].cpu().numpy(), row["loss_trace"], rtol=1e-9)
