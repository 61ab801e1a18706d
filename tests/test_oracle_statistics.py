"""Monte Carlo error of the population estimator (Sec. 2.4 step 7 and the
error study of Sec. 3): the standard error that one ensemble reports matches
the spread of its population estimate over independent seeds, and it falls
as N^(-1/2).

QCLE crossing (Sec. 3.3), 1-D, 12 independent seeds at N = 64 and N = 256
beams, the real parts of the upper and lower populations and of the
coherence u21.  With 11 degrees of freedom, the ratio of the empirical
spread to the reported error lies in [0.49, 1.56] with probability 0.99;
the ratio of the errors at N = 64 and N = 256 is 2 up to the scatter of
the error estimates themselves ([1.6, 2.5]).  The seeds are fixed, so the
test is deterministic.
"""

import numpy as np
import pytest

from oracle import models, observables, sampling, shgb

PAR = dict(A=0.01, B=1.6, C=0.005, D=1.0, mass=2000.0)
EPS = 0.01
SEEDS = [1703 + 17 * k for k in range(12)]


def estimate(n, seed):
    mdl = models.QCLE(**PAR)
    ens = sampling.init_beams(mdl, n, EPS, seed, -0.6, 0.3, "normal", 30.0, 1.0, 1)
    shgb.advance(mdl, ens, 150, 0.5, seed)
    mean, se = observables.population_mean_se(observables.populations(ens, EPS), n)
    return mean, se


@pytest.fixture(scope="module")
def runs():
    return {n: [estimate(n, s) for s in SEEDS] for n in (64, 256)}


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_reported_error_matches_spread_over_seeds(runs, comp):
    for n, res in runs.items():
        means = np.array([m[comp].real for m, _ in res])
        se = np.array([s[comp].real for _, s in res])
        spread = means.std(ddof=1)
        reported = np.sqrt((se ** 2).mean())
        assert reported > 0
        print(f"N={n} comp={comp}: spread / reported error = {spread / reported:.3f}")
        assert 0.49 <= spread / reported <= 1.56, (n, comp, spread, reported)


def test_error_falls_as_inverse_square_root(runs):
    for comp in (1, 2):
        r = [np.sqrt((np.array([s[comp].real for _, s in runs[n]]) ** 2).mean()) for n in (64, 256)]
        print(f"comp={comp}: error ratio N=64 / N=256 = {r[0] / r[1]:.3f}")
        assert 1.6 <= r[0] / r[1] <= 2.5, (comp, r)
