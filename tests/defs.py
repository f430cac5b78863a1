"""Definitions written out again in numpy, straight from the paper, to pin the
oracle (test helpers only; no code shared with the oracle or the GPU library).

Site i = x + L*(y + L*z); J[d][i] is the bond between i and i + e_d.
"""
from __future__ import annotations

import numpy as np
from scipy import stats


def grid(a: np.ndarray, L: int) -> np.ndarray:
    """Flat site array -> [z][y][x] view."""
    return a.reshape(a.shape[:-1] + (L, L, L))


def energy(spins: np.ndarray, J: np.ndarray, L: int) -> np.ndarray:
    """H = -sum over the 3V bonds of J_ij s_i s_j (paper Eq. 1).  spins [..., V]."""
    s = grid(spins.astype(np.float64), L)
    Jg = grid(np.asarray(J, dtype=np.float64), L)
    e = 0.0
    for d, axis in ((0, -1), (1, -2), (2, -3)):
        e = e - (Jg[d] * s * np.roll(s, -1, axis=axis)).sum(axis=(-1, -2, -3))
    return e


def overlaps(sa: np.ndarray, sb: np.ndarray, L: int) -> tuple[int, int]:
    """Q = sum_i q_i and Q_l = sum over the 3V bonds of q_i q_j (Eqs. 2-4)."""
    q = grid((sa.astype(np.int64) * sb.astype(np.int64)), L)
    Q = int(q.sum())
    QL = int(sum((q * np.roll(q, -1, axis=ax)).sum() for ax in (-1, -2, -3)))
    return Q, QL


def all_states(V: int) -> np.ndarray:
    """All 2^V configurations; state index g has s_i = -1 iff bit i of g is set."""
    g = np.arange(2 ** V, dtype=np.int64)[:, None]
    bits = (g >> np.arange(V)) & 1
    return (1 - 2 * bits).astype(np.int8)


def state_index(spins: np.ndarray) -> np.ndarray:
    bits = (np.asarray(spins) < 0).astype(np.int64)
    return (bits << np.arange(bits.shape[-1])).sum(axis=-1)


def boltzmann(J: np.ndarray, L: int, beta: float) -> np.ndarray:
    states = all_states(L ** 3)
    E = energy(states, J, L)
    w = np.exp(-beta * (E - E.min()))
    return w / w.sum()


def sweep_kernel(J: np.ndarray, L: int, beta: float, rule: str = "metropolis") -> np.ndarray:
    """Exact transition matrix of one checkerboard sweep: sites of parity 0 in
    increasing order, then parity 1, each flipped with probability
    min{1, exp(-beta dH)} (Metropolis, paper Sec. 3 and App. A.1) or
    1 / (1 + exp(beta dH)) (heat bath: the spin drawn from its conditional
    Boltzmann weight), dH = H(flipped) - H."""
    V = L ** 3
    states = all_states(V)
    E = energy(states, J, L)
    n = 2 ** V
    x, y, z = np.arange(V) % L, (np.arange(V) // L) % L, np.arange(V) // (L * L)
    order = [i for p in (0, 1) for i in range(V) if (x[i] + y[i] + z[i]) % 2 == p]
    P = np.eye(n)
    idx = np.arange(n)
    for i in order:
        flipped = idx ^ (1 << i)
        dH = E[flipped] - E
        if rule == "metropolis":
            acc = np.minimum(1.0, np.exp(-beta * dH))
        else:
            acc = 1.0 / (1.0 + np.exp(beta * dH))
        K = np.zeros((n, n))
        K[idx, flipped] = acc
        K[idx, idx] = 1.0 - acc
        P = P @ K
    return P


def micsa_kernel(J: np.ndarray, L: int, beta: float, n_sweeps: int) -> np.ndarray:
    """Exact transition matrix of one MicSA period (App. A.1): a walker drawn
    from its Boltzmann law (density beta exp(-beta W), W >= 0), then n_sweeps
    sweeps in the checkerboard order in which each spin flips iff the walker
    holds at least dH, which the walker then gives up.  Given the state the
    period is a deterministic function of the drawn W0, piecewise constant:
    every test W0 - (energy given up so far) >= dH splits the current interval
    of W0 at one threshold, and a final state collects the probability
    exp(-beta a) - exp(-beta b) of each interval [a, b) leading to it."""
    V = L ** 3
    states = all_states(V)
    E = energy(states, J, L)
    n = 2 ** V
    x, y, z = np.arange(V) % L, (np.arange(V) // L) % L, np.arange(V) // (L * L)
    order = [i for p in (0, 1) for i in range(V) if (x[i] + y[i] + z[i]) % 2 == p] * n_sweeps
    P = np.zeros((n, n))
    for g0 in range(n):
        pieces = [(0.0, np.inf, g0, 0.0)]  # W0 in [a, b), state, energy given up
        for i in order:
            nxt = []
            for a, b, g, c in pieces:
                f = g ^ (1 << i)
                th = E[f] - E[g] + c  # accept iff W0 >= th
                if th <= a:
                    nxt.append((a, b, f, c + E[f] - E[g]))
                elif th >= b:
                    nxt.append((a, b, g, c))
                else:
                    nxt.append((a, th, g, c))
                    nxt.append((th, b, f, c + E[f] - E[g]))
            pieces = nxt
        for a, b, g, _ in pieces:
            P[g0, g] += np.exp(-beta * a) - (0.0 if np.isinf(b) else np.exp(-beta * b))
    return P


def chi2_pvalue(counts: np.ndarray, probs: np.ndarray, min_expected: float = 5.0) -> float:
    """Pearson chi-square goodness of fit, pooling cells with small expectation."""
    counts = np.asarray(counts, dtype=np.float64)
    n = counts.sum()
    exp = probs * n
    big = exp >= min_expected
    obs_c = list(counts[big])
    exp_c = list(exp[big])
    if (~big).any():
        obs_c.append(counts[~big].sum())
        exp_c.append(exp[~big].sum())
    obs_c, exp_c = np.array(obs_c), np.array(exp_c)
    keep = exp_c > 0
    stat = ((obs_c[keep] - exp_c[keep]) ** 2 / exp_c[keep]).sum()
    dof = max(int(keep.sum()) - 1, 1)
    return float(stats.chi2.sf(stat, dof))


def cluster_stats(labels: np.ndarray, sa: np.ndarray, sb: np.ndarray, top: int = 6) -> np.ndarray:
    """Sizes of the `top` largest clusters of the majority and of the minority
    (paper Sec. 1, Fig. 1): clusters are the connected components of equal site
    overlap q_i = s_i^a s_i^b given by `labels` (one id per site); the majority
    are the clusters whose q_i has the sign of q = sum_i q_i (q >= 0 counted
    as positive).  Returns int [2][top], descending, 0-padded."""
    q = sa.astype(np.int64) * sb.astype(np.int64)
    maj = 1 if q.sum() >= 0 else -1
    out = np.zeros((2, top), dtype=np.int64)
    ids, first, counts = np.unique(labels, return_index=True, return_counts=True)
    sign = q[first]
    for row, want in ((0, maj), (1, -maj)):
        sizes = np.sort(counts[sign == want])[::-1][:top]
        out[row, :len(sizes)] = sizes
    return out
