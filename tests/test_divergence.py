"""Divergence status (Sec. 2.1, eq. 2's step size alpha), host side: the
library's rule applied to residual sequences of the FP64 oracle's Landweber
iteration.  p A^T A is positive semi-definite with largest eigenvalue
lambda, so for alpha <= 2/lambda the residual cannot grow; beyond it the
component along the top eigenvector grows by |1 - alpha lambda| per step."""

import math

import numpy as np
import pytest

import oracle
import paper_2103_10329_amd as mg
from conftest import random_views


@pytest.fixture(scope="module")
def lib():
    import os
    if not os.path.exists(mg.LIB_PATH):
        from paper_2103_10329_amd import build
        build.build()
    return mg.load_library()


def _residuals(alpha_factor, steps=12, kind="identity"):
    rng = np.random.Generator(np.random.PCG64(77))
    views = random_views(rng, 10, radius=14.0, det_dist=10.0, pixel=1.2, allow_z=False)
    g = oracle.Geom(6, 6, 6, 1.0, (0, 0, 0), 7, 7, views)
    b = rng.random(g.stack_shape)   # inconsistent data
    filt = {"identity": oracle.filter_identity(), "stencil27": oracle.filter_stencil27()}[kind]
    lam = oracle.power_iteration(g, filt, iters=200)
    mu = np.zeros(g.vol_shape)
    res = []
    for _ in range(steps):
        mu, r = oracle.landweber_step(g, mu, b, alpha_factor / lam, filt)
        res.append(r)
    return res


def _first_flag(res, ratio):
    for k in range(1, len(res)):
        if mg.residual_diverged(res[k - 1], res[k], ratio):
            return k
    return None


def test_rule_by_hand(lib):
    assert mg.residual_diverged(1.0, 1.06, 1.05)
    assert not mg.residual_diverged(1.0, 1.04, 1.05)
    assert mg.residual_diverged(1.0, math.nan, 1.05)
    assert mg.residual_diverged(1.0, math.inf, 0.0)
    assert not mg.residual_diverged(1.0, 100.0, 0.0)    # ratio 0: finiteness only
    assert not mg.residual_diverged(0.0, 5.0, 1.05)     # no previous residual


@pytest.mark.parametrize("kind", ["identity", "stencil27"])
def test_stable_step_never_flags(lib, kind):
    res = _residuals(1.0, kind=kind)
    assert _first_flag(res, 1.05) is None
    assert all(res[k + 1] <= res[k] * (1 + 1e-12) for k in range(len(res) - 1))


@pytest.mark.parametrize("kind", ["identity", "stencil27"])
def test_step_beyond_two_over_lambda_is_flagged(lib, kind):
    res = _residuals(4.0, kind=kind)       # |1 - alpha lambda| = 3 on the top eigenvector
    k = _first_flag(res, 1.05)
    assert k is not None and k <= 8, res
