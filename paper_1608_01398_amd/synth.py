"""Seeded synthetic GWAS inputs: HWE genotypes packed as PLINK 1 .bed rows, traits and covariates.

This module is shared by the tests, the benchmark and the smoke run as the single source of
inputs for both the oracle and the device path. It holds none of the IHT method's arithmetic:
phenotypes are built from the *population* allele frequency q_j that the generator itself drew
(standardising by 2q_j and sqrt(2q_j(1-q_j))), never from the sample mean/precision that the
method computes.

Workload shape follows the paper's data (Results, NFBC1966: a few thousand subjects by a few
hundred thousand SNPs, PLINK-compressed, with missing genotypes and non-genetic covariates);
the real cohort is controlled-access, so every input here is synthetic.

PLINK 1 SNP-major layout: SNP j occupies ``row_bytes = ceil(n/4)`` bytes; subject i sits in byte
``i // 4`` at bits ``2*(i % 4)`` (low pair first). Two-bit values: 0 = homozygous first allele,
1 = missing, 2 = heterozygous, 3 = homozygous second allele. Pad bits past n are 0.
"""
from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

# PLINK two-bit values
CODE_HOM_A1, CODE_MISSING, CODE_HET, CODE_HOM_A2 = 0, 1, 2, 3

# Shapes of the standard workloads (subjects n, SNPs p, causal count, effect range, fitted k,
# number of dense N(0,1) covariates, intercept value of the trait).
CONFIGS = {
    "c1": dict(n=1000, p=10_000, k_true=10, eff=(0.2, 0.5), k=10, covariates=0, intercept=0.0),
    "c2": dict(n=5000, p=500_000, k_true=20, eff=(0.1, 0.4), k=20, covariates=0, intercept=0.0),
    "c4": dict(n=10_000, p=1_000_000, k_true=20, eff=(0.1, 0.4), k=20, covariates=0, intercept=0.0),
    "c5": dict(n=20_000, p=2_000_000, k_true=100, eff=(0.05, 0.3), k=100, covariates=5, intercept=1.0),
}

MAF_RANGE = (0.05, 0.5)
MISSING_RATE = 0.01
_BLOCK = 2048


def row_bytes(n: int) -> int:
    return (n + 3) // 4


def pack_codes(codes: np.ndarray) -> np.ndarray:
    """Pack a [p, n] array of two-bit PLINK values into [p, ceil(n/4)] bytes (low pair first)."""
    codes = np.asarray(codes, dtype=np.uint8)
    p, n = codes.shape
    rb = row_bytes(n)
    padded = np.zeros((p, rb * 4), dtype=np.uint8)
    padded[:, :n] = codes & 3
    q = padded.reshape(p, rb, 4)
    return (q[:, :, 0] | (q[:, :, 1] << 2) | (q[:, :, 2] << 4) | (q[:, :, 3] << 6)).astype(np.uint8)


def unpack_codes(bed: np.ndarray, n: int) -> np.ndarray:
    """Inverse of :func:`pack_codes`: [p, row] bytes -> [p, n] two-bit values."""
    bed = np.asarray(bed, dtype=np.uint8)
    p = bed.shape[0]
    out = np.empty((p, bed.shape[1] * 4), dtype=np.uint8)
    for t in range(4):
        out[:, t::4] = (bed >> (2 * t)) & 3
    return out[:, :n]


def _gen_block(args):
    seed, block, n, q, miss = args
    rng = np.random.Generator(np.random.PCG64([seed, 7, block]))
    b = q.shape[0]
    u = rng.random((b, n), dtype=np.float32)
    qq = q.astype(np.float64)[:, None]
    t0 = np.float32(miss)
    t1 = (miss + (1.0 - miss) * (1.0 - qq) ** 2).astype(np.float32)
    t2 = (t1 + (1.0 - miss) * 2.0 * qq * (1.0 - qq)).astype(np.float32)
    k = (u >= t0).astype(np.uint8) + (u >= t1) + (u >= t2)
    # k: 0 -> missing, 1 -> hom A1, 2 -> het, 3 -> hom A2 (A2 frequency q: the counted allele)
    lut = np.array([CODE_MISSING, CODE_HOM_A1, CODE_HET, CODE_HOM_A2], dtype=np.uint8)
    return block, pack_codes(lut[k])


def make_genotypes(n: int, p: int, seed: int, miss: float = MISSING_RATE, maf=MAF_RANGE, workers: int | None = None):
    """HWE genotypes: q_j ~ U(maf), dosage ~ Binomial(2, q_j), each entry missing with prob ``miss``.

    Returns (bed [p, ceil(n/4)] uint8, q [p] float64). Deterministic in (n, p, seed, miss, maf)
    regardless of the worker count.
    """
    rng = np.random.Generator(np.random.PCG64([seed, 1]))
    q = rng.uniform(maf[0], maf[1], size=p)
    rb = row_bytes(n)
    bed = np.empty((p, rb), dtype=np.uint8)
    nblocks = (p + _BLOCK - 1) // _BLOCK
    jobs = [(seed, b, n, q[b * _BLOCK:(b + 1) * _BLOCK], miss) for b in range(nblocks)]
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    if workers <= 1 or n * p < 50_000_000:
        for job in jobs:
            b, packed = _gen_block(job)
            bed[b * _BLOCK:b * _BLOCK + packed.shape[0]] = packed
    else:
        with ProcessPoolExecutor(max_workers=workers) as ex:
            for b, packed in ex.map(_gen_block, jobs, chunksize=4):
                bed[b * _BLOCK:b * _BLOCK + packed.shape[0]] = packed
    return bed, q


def _population_standardized(bed: np.ndarray, n: int, q: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """Columns ``cols`` scaled by population frequency: (dose - 2q)/sqrt(2q(1-q)); missing -> 0."""
    codes = unpack_codes(bed[cols], n).astype(np.int64)
    dose = np.select([codes == CODE_HOM_A1, codes == CODE_HET, codes == CODE_HOM_A2], [0, 1, 2], default=-1)
    qc = q[cols][:, None]
    z = (dose - 2.0 * qc) / np.sqrt(2.0 * qc * (1.0 - qc))
    z[dose < 0] = 0.0
    return z.T  # [n, len(cols)]


def make_covariates(n: int, c: int, seed: int) -> np.ndarray:
    """Dense N(0,1) non-genetic covariates, float32, column-major [n x c] (as an [c, n] array)."""
    rng = np.random.Generator(np.random.PCG64([seed, 3]))
    return rng.standard_normal((c, n)).astype(np.float32)


def make_trait(bed: np.ndarray, n: int, q: np.ndarray, k_true: int, eff, seed: int,
               Z: np.ndarray | None = None, intercept: float = 0.0, noise: float = 1.0):
    """y = sum_l beta_l z_l + Z gamma + intercept + N(0, noise^2).

    Causal positions are uniform without replacement; effects are +-U(eff) with equiprobable sign;
    covariate effects gamma_c are +-U(0.1, 0.5). Returns (y float64 [n], causal idx, beta, gamma).
    """
    p = bed.shape[0]
    rng = np.random.Generator(np.random.PCG64([seed, 2]))
    causal = np.sort(rng.choice(p, size=k_true, replace=False))
    beta = rng.uniform(eff[0], eff[1], size=k_true) * rng.choice([-1.0, 1.0], size=k_true)
    y = _population_standardized(bed, n, q, causal) @ beta
    gamma = np.zeros(0)
    if Z is not None and Z.shape[0] > 0:
        gamma = rng.uniform(0.1, 0.5, size=Z.shape[0]) * rng.choice([-1.0, 1.0], size=Z.shape[0])
        y = y + Z.astype(np.float64).T @ gamma
    y = y + intercept + noise * rng.standard_normal(n)
    return y, causal, beta, gamma


def make_binary_trait(bed: np.ndarray, n: int, q: np.ndarray, k_true: int, eff, seed: int, intercept: float = -0.5):
    """Case/control trait: y_i ~ Bernoulli(1 / (1 + exp(-(sum_l beta_l z_l + intercept)))) with the
    causal columns and effects drawn as in make_trait. Returns (y float64 0/1 [n], causal, beta)."""
    p = bed.shape[0]
    rng = np.random.Generator(np.random.PCG64([seed, 5]))
    causal = np.sort(rng.choice(p, size=k_true, replace=False))
    beta = rng.uniform(eff[0], eff[1], size=k_true) * rng.choice([-1.0, 1.0], size=k_true)
    eta = _population_standardized(bed, n, q, causal) @ beta + intercept
    y = (rng.random(n) < 1.0 / (1.0 + np.exp(-eta))).astype(np.float64)
    return y, causal, beta


def make_subset(n: int, size: int, seed: int) -> np.ndarray:
    """A random subject subset of the given size as a 0/1 uint8 mask of length n."""
    rng = np.random.Generator(np.random.PCG64([seed, 4]))
    m = np.zeros(n, dtype=np.uint8)
    m[rng.choice(n, size=size, replace=False)] = 1
    return m


def make_folds(n: int, q: int, seed: int) -> np.ndarray:
    """Seeded balanced partition of n subjects into q folds: uint8 [n] fold index of each subject."""
    return np.random.default_rng(seed).permutation(np.arange(n) % q).astype(np.uint8)


def mask_to_bits(mask: np.ndarray) -> np.ndarray:
    """0/1 per-subject mask -> packed little-endian bit array (bit i%8 of byte i//8)."""
    return np.packbits(np.asarray(mask, dtype=np.uint8), bitorder="little")


def make_problem(cfg: str, seed: int, n: int | None = None, p: int | None = None, workers: int | None = None):
    """Full synthetic problem for a named workload, optionally with n/p overridden."""
    c = dict(CONFIGS[cfg])
    if n is not None:
        c["n"] = n
    if p is not None:
        c["p"] = p
    bed, q = make_genotypes(c["n"], c["p"], seed, workers=workers)
    Z = make_covariates(c["n"], c["covariates"], seed) if c["covariates"] else None
    y, causal, beta, gamma = make_trait(bed, c["n"], q, min(c["k_true"], c["p"]), c["eff"], seed, Z=Z,
                                        intercept=c["intercept"])
    return dict(cfg=cfg, seed=seed, n=c["n"], p=c["p"], k=c["k"], bed=bed, q=q, y=y, Z=Z,
                causal=causal, beta_true=beta, gamma_true=gamma)
