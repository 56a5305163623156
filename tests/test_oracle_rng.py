"""Pins of the oracle's Philox4x32-10 generator.

The generator is pinned against rocRAND's Philox4x32-10 (a separate, public
implementation of the same SC'11 definition) run as a black box on the host,
and its uniform-float mapping against a chi-square test.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest


def _hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return None


def _rocrand_outputs(triples):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available to build the rocRAND host check")
    src = os.path.join(os.path.dirname(__file__), "philox_rocrand_check.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "philox_check")
        subprocess.check_call([hipcc, "-O1", "-o", exe, src])
        text = "\n".join("%d %d %d" % t for t in triples) + "\n"
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    return np.array([[int(w, 16) for w in line.split()] for line in out.strip().splitlines()],
                    dtype=np.uint32)


def test_philox_matches_rocrand(orc):
    # rocRAND state (seed, subsequence, offset) is counter
    # (offset/4 lo, offset/4 hi, subsequence lo, subsequence hi) under key
    # (seed lo, seed hi); cover every counter and key word.
    rng = np.random.default_rng(7)
    triples, ctrs, keys = [], [], []
    for i in range(24):
        seed = int(rng.integers(0, 2**63)) if i else 0
        sub = int(rng.integers(0, 2**63)) if i % 3 else int(rng.integers(0, 2**32))
        blk = int(rng.integers(0, 2**62)) if i % 2 else int(rng.integers(0, 2**16))
        triples.append((seed, sub, 4 * blk))
        ctrs.append([blk & 0xFFFFFFFF, blk >> 32, sub & 0xFFFFFFFF, sub >> 32])
        keys.append([seed & 0xFFFFFFFF, seed >> 32])
    ref = _rocrand_outputs(triples)
    mine = np.stack([orc.philox(np.array([c], np.uint64).astype(np.uint32), np.array(k, np.uint64).astype(np.uint32))[0]
                     for c, k in zip(ctrs, keys)])
    np.testing.assert_array_equal(mine, ref)


def test_unit_float_uniformity(orc):
    # the cluster draw uses the top 24 bits of word 0 as u in [0,1): check
    # uniformity over 64 bins with chi-square (p > 1e-4 at 63 dof: < 120)
    n = 1 << 16
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n)
    ctr[:, 2] = 5
    w = orc.philox(ctr, [123, 456])
    u = (w[:, 0] >> 8).astype(np.float64) / 2**24
    assert u.min() >= 0.0 and u.max() < 1.0
    h, _ = np.histogram(u, bins=64, range=(0.0, 1.0))
    e = n / 64
    chi2 = float(((h - e) ** 2 / e).sum())
    assert chi2 < 120.0, chi2
    # consecutive counters decorrelated
    c = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(c) < 0.03
