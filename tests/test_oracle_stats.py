"""Distributional pins of the oracle's sampling against the closed forms of the
toy shower model (Kolmogorov-Smirnov and binomial tests, fixed seeds).

* bremsstrahlung photon energy k ~ 1/k on [1 MeV, E]: ln k / ln E is uniform;
* pair production: the electron's share of the kinetic energy is uniform;
* first interaction of a photon inside the 2.3 mm absorber of layer 0:
  probability 1 - exp(-2.3 / lambda) with lambda = 9/7 X0 = 7.2 mm (pair) or
  2 X0 = 11.2 mm (Compton);
* multiple scattering: the space angle after one step is Rayleigh(theta0) with
  theta0 = 13.6 / E * sqrt(s / X0), and the azimuth is uniform.
"""
import math

import numpy as np
import pytest
from scipy import stats

import workloads

N = 20000


def run_one_iteration(oracle_mod, ptype, E, nl, precision=0, n=N, seed=3):
    o = oracle_mod.Oracle(oracle_mod.DENSE, precision, 1 << 16, [seed])
    p = workloads.primaries(n, ptype, E, num_ia_left=nl)
    assert o.inject(p) == 0
    rc, _ = o.step()
    assert rc == 0
    return o


@pytest.mark.parametrize("precision", [0, 1])
def test_brem_spectrum(oracle_mod, precision):
    o = run_one_iteration(oracle_mod, workloads.ELECTRON, 100.0, 1e-9, precision)
    g, _ = o.dump(workloads.GAMMA)
    e, _ = o.dump(workloads.ELECTRON)
    assert len(g) == N  # every electron radiated once at its first step
    E1 = 100.0 - 1.27 * (1e-9 * 5.6)
    u = np.log(g["E"]) / math.log(E1)
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    assert abs(g["E"].mean() - (E1 - 1) / math.log(E1)) < 5 * g["E"].std() / math.sqrt(N)
    # energy is shared exactly between the photon and the surviving electron
    surv = {int(t): float(x) for t, x in zip(e["trackId"], e["E"])}
    for k in range(200):
        parent = int(g[k]["parentId"])
        if parent in surv:
            assert surv[parent] + g[k]["E"] == (np.float32(E1) if precision else E1)


@pytest.mark.parametrize("precision", [0, 1])
def test_pair_split_uniform(oracle_mod, precision):
    o = run_one_iteration(oracle_mod, workloads.GAMMA, 50.0, 1e-9, precision)
    e, _ = o.dump(workloads.ELECTRON)
    T = 50.0 - 1.022
    # conditioned on being buffered (T- >= 1 MeV) the electron share is uniform on [1, T]
    u = (e["E"] - 1.0) / (T - 1.0)
    assert len(e) > 0.9 * N
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    p, _ = o.dump(workloads.POSITRON)
    assert len(p) > 0.9 * N


@pytest.mark.parametrize("E,lam", [(100.0, 7.2), (0.5, 11.2)])
def test_first_interaction_probability(oracle_mod, E, lam):
    o = run_one_iteration(oracle_mod, workloads.GAMMA, E, -1.0)
    g, _ = o.dump(workloads.GAMMA)
    crossed = int(np.sum(g["volume"] == 1))
    p_hat = 1.0 - crossed / N
    p = 1.0 - math.exp(-2.3 / lam)
    assert abs(p_hat - p) < 5 * math.sqrt(p * (1 - p) / N)


@pytest.mark.parametrize("precision", [0, 1])
def test_msc_rayleigh(oracle_mod, precision):
    o = run_one_iteration(oracle_mod, workloads.ELECTRON, 100.0, 1e9, precision)
    e, _ = o.dump(workloads.ELECTRON)
    assert len(e) == N and np.all(e["volume"] == 1)
    th0 = 13.6 / 100.0 * math.sqrt(2.3 / 5.6)
    d = e["dir"]
    theta = np.arctan2(np.hypot(d[:, 0], d[:, 1]), d[:, 2])
    cdf = lambda x: 1.0 - np.exp(-(x**2) / (2 * th0**2))
    assert stats.kstest(theta, cdf).pvalue > 1e-3
    phi = (np.arctan2(d[:, 1], d[:, 0]) + 2 * math.pi) % (2 * math.pi)
    assert stats.kstest(phi / (2 * math.pi), "uniform").pvalue > 1e-3
