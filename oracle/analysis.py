"""Production analysis written from the definitions -- TEST INFRASTRUCTURE.

  * ``jackknife_log_dos``: ln g from the summed block histograms (Sec. 2.1,
    Sec. 3.3) and, per bin, the jackknife error over the blocks: with x_(b)
    the estimate from all blocks but b and x_. their mean,
    err = sqrt((B-1)/B * sum_b (x_(b) - x_.)^2);
  * ``canonical``: <E>/N and beta^2 Var(E)/N at inverse temperature beta
    from ln g, P_beta(E) ~ g(E) exp(-beta E) (Sec. 2.1);
  * ``canonical_jackknife``: the same from block histograms, with jackknife
    errors;
  * ``brute_force_canonical`` and ``transfer_matrix_canonical``: the same
    canonical averages computed without any density of states, as pins.
"""
import math

import numpy as np

from . import log_dos


def _loo_histograms(block_hists):
    h = np.asarray(block_hists, dtype=np.uint64)
    total = h.sum(axis=0, dtype=np.uint64)
    return total, [total - h[b] for b in range(h.shape[0])]


def _jk(values):
    v = np.asarray(values, dtype=np.float64)
    B = v.shape[0]
    if B < 2:
        return np.zeros(v.shape[1:])
    mean = v.mean(axis=0)
    return np.sqrt((B - 1) / B * ((v - mean) ** 2).sum(axis=0))


def jackknife_log_dos(block_hists, omega, norm=1):
    total, loo = _loo_histograms(block_hists)
    est = log_dos(total, omega, norm)
    B = len(loo)
    err = np.full(est.shape, np.nan)
    if B < 2:
        err[np.isfinite(est)] = 0.0
        return est, err
    samples = [log_dos(h, omega, norm) for h in loo]
    for k in range(est.size):
        if not np.isfinite(est[k]):
            continue
        col = [s[k] for s in samples]
        if not all(np.isfinite(col)):
            err[k] = np.inf
            continue
        err[k] = float(_jk(np.array(col)[:, None])[0])
    return est, err


def canonical(ln_g, betas):
    """(energy per spin, specific heat per spin) at each beta."""
    ln_g = np.asarray(ln_g, dtype=np.float64)
    N = ln_g.size - 1
    E = 4.0 * np.arange(N + 1) - 2.0 * N
    ok = np.isfinite(ln_g)
    es, cs = [], []
    for beta in np.atleast_1d(betas):
        a = ln_g[ok] - beta * E[ok]
        p = np.exp(a - a.max())
        z = p.sum()
        m1 = (p * E[ok]).sum() / z
        m2 = (p * E[ok] ** 2).sum() / z
        es.append(m1 / N)
        cs.append(beta * beta * (m2 - m1 * m1) / N)
    return np.array(es), np.array(cs)


def canonical_jackknife(block_hists, omega, betas):
    total, loo = _loo_histograms(block_hists)
    e, c = canonical(log_dos(total, omega, 1), betas)
    if len(loo) < 2:
        return e, np.zeros_like(e), c, np.zeros_like(c)
    le, lc = zip(*[canonical(log_dos(h, omega, 1), betas) for h in loo])
    return e, _jk(np.array(le)), c, _jk(np.array(lc))


def brute_force_canonical(L, betas):
    """<E>/N and beta^2 Var(E)/N by summing over all 2^(L*L) states."""
    N = L * L
    if N > 20:
        raise ValueError("brute force only for L = 4")
    states = np.arange(1 << N, dtype=np.int64)
    spins = ((states[:, None] >> np.arange(N)) & 1) * 2 - 1
    s = spins.reshape(-1, L, L)
    energy = -(s * np.roll(s, -1, axis=2)).sum(axis=(1, 2)) - (s * np.roll(s, -1, axis=1)).sum(axis=(1, 2))
    energy = energy.astype(np.float64)
    es, cs = [], []
    for beta in np.atleast_1d(betas):
        a = -beta * energy
        p = np.exp(a - a.max())
        z = p.sum()
        m1 = (p * energy).sum() / z
        m2 = (p * energy ** 2).sum() / z
        es.append(m1 / N)
        cs.append(beta * beta * (m2 - m1 * m1) / N)
    return np.array(es), np.array(cs)


def _ln_z_transfer(L, beta):
    """ln Z of the periodic L x L lattice as ln Tr(T^L), T the symmetric
    row-to-row transfer matrix, from its eigenvalues."""
    rows = np.arange(1 << L)
    s = ((rows[:, None] >> np.arange(L)) & 1) * 2 - 1
    e_row = -(s * np.roll(s, -1, axis=1)).sum(axis=1).astype(np.float64)
    e_inter = -(s @ s.T).astype(np.float64)
    t = np.exp(-beta * (0.5 * e_row[:, None] + e_inter + 0.5 * e_row[None, :]))
    lam = np.linalg.eigvalsh(t)
    lmax = np.max(np.abs(lam))
    return L * math.log(lmax) + math.log(np.sum((lam / lmax) ** L))


def transfer_matrix_canonical(L, beta, h=1e-3):
    """<E>/N and beta^2 Var(E)/N from ln Z(beta) by central differences
    (fourth-order stencils): <E> = -d lnZ/d beta, Var(E) = d^2 lnZ/d beta^2."""
    N = L * L
    f = [_ln_z_transfer(L, beta + j * h) for j in (-2, -1, 0, 1, 2)]
    d1 = (f[0] - 8 * f[1] + 8 * f[3] - f[4]) / (12 * h)
    d2 = (-f[0] + 16 * f[1] - 30 * f[2] + 16 * f[3] - f[4]) / (12 * h * h)
    return -d1 / N, beta * beta * d2 / N
