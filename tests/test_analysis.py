"""The analysis layer (log2 bins, disorder averages, SDY test, P(q) moments,
round-trip time): known answers on synthetic snapshots, and a logged oracle
run whose bin averages are recomputed EMCS by EMCS."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2605_25872_amd import analysis, inputs


class OracleRunner:
    """The oracle behind the interface run_logged expects of a context."""

    def __init__(self, o):
        self.o = o

    def set_schedule(self, **kw):
        pass

    def new_obs(self):
        return self.o.new_observables()

    def run(self, n, obs):
        self.o.run(n, obs)

    def obs_arrays(self, obs):
        return {"n_meas": int(obs.n_meas[0]), "acc": obs.acc, "hist": obs.hist}

    def read_pt(self):
        return {"rt_count": self.o.rt_count.copy()}


def test_log2_bins_follow_the_definition():
    """bin(b) = [t_max/2^(b+1) + 1, t_max/2^b]: bin 0 is the second half, bin 1
    the second quarter, ... (Sec. 4, Eq. 8)."""
    assert analysis.log2_bins(16) == [(9, 16), (5, 8), (3, 4), (2, 2), (1, 1)]
    assert analysis.log2_bins(16, 2) == [(9, 16), (5, 8)]
    assert analysis.snapshot_times(16) == [0, 1, 2, 4, 8, 16]
    t_max = 38_400_000  # the paper's L=16 run
    bins = analysis.log2_bins(t_max, 4)
    assert bins[0] == (t_max // 2 + 1, t_max) and bins[3] == (t_max // 16 + 1, t_max // 8)
    for (lo0, hi0), (lo1, hi1) in zip(bins, bins[1:]):
        assert hi1 == lo0 - 1  # contiguous, going back in time
    assert analysis.log2_bins(12) == [(7, 12), (4, 6), (2, 3), (1, 1)]
    with pytest.raises(ValueError):
        analysis.log2_bins(0)


def _snap(t, acc, hist, rt):
    return analysis.Snapshot(t, t, np.asarray(acc, float), np.asarray(hist, np.uint64), np.asarray(rt, np.uint64))


def test_bin_averages_on_synthetic_snapshots():
    """Two samples, two temperatures, N_r = 3 (3 pairs), V = 2: averages per
    replica or pair, sample-to-sample errors, Binder ratio, normalised P(q) and
    tau_TRW = N_r N_T EMCS / round trips."""
    S, NT, NR, V = 2, 2, 3, 2
    n = 4  # EMCS in the bin
    a0 = np.zeros((S, NT, 6))
    a1 = np.zeros((S, NT, 6))
    e = np.array([[-1.5, -1.0], [-1.3, -0.8]])      # per-replica mean energy per spin
    q2 = np.array([[0.5, 0.2], [0.7, 0.1]])
    q4 = np.array([[0.4, 0.1], [0.6, 0.05]])
    sdy = np.array([[0.02, -0.01], [0.04, 0.03]])
    a1[..., 0] = e * NR * n
    a1[..., 1] = e ** 2 * NR * n
    a1[..., 2] = q2 * 3 * n
    a1[..., 3] = q4 * 3 * n
    a1[..., 4] = 0.5 * 3 * n
    a1[..., 5] = sdy * 3 * n
    h0 = np.zeros((NT, V + 1))
    h1 = np.array([[2, 0, 6], [1, 2, 1]])
    T = np.array([0.5, 1.0])
    r = analysis.bin_result(_snap(10, a0, h0, [5, 7]), _snap(10 + n, a1, h1, [7, 7]), 0, T, NR)
    assert (r.lo, r.hi, r.n_emcs) == (11, 14, 4)
    np.testing.assert_allclose(r.per_sample["e"], e)
    np.testing.assert_allclose(r.e, e.mean(axis=0))
    np.testing.assert_allclose(r.e_err, e.std(axis=0, ddof=1) / np.sqrt(2))
    np.testing.assert_allclose(r.sdy, sdy.mean(axis=0))
    np.testing.assert_allclose(r.q2, q2.mean(axis=0))
    np.testing.assert_allclose(r.binder, 0.5 * (3 - q4.mean(axis=0) / q2.mean(axis=0) ** 2))
    np.testing.assert_allclose(r.pq, [[0.25, 0.0, 0.75], [0.25, 0.5, 0.25]])
    np.testing.assert_allclose(r.round_trips, [2, 0])
    assert r.tau_trw[0] == NR * NT * n / 2 and np.isinf(r.tau_trw[1])
    assert r.round_trips_per_clone_median(NR * NT) == pytest.approx(np.median([2 / 6, 0]))
    # SDY: positive by more than 2 errors means not equilibrated
    z = r.sdy / r.sdy_err
    np.testing.assert_allclose(r.sdy_z(), z)
    np.testing.assert_array_equal(r.sdy_equilibrated(2.0), z <= 2.0)
    with pytest.raises(ValueError):
        analysis.bin_result(_snap(3, a0, h0, [0, 0]), _snap(3, a1, h1, [0, 0]), 0, T, NR)


def test_logged_oracle_run_matches_per_emcs_measurements():
    """run_logged + analyse on the oracle equal the averages of observables
    measured EMCS by EMCS over each bin (a second, identical oracle), and the
    round trips per bin equal the counts' increments."""
    L, S, NR, NT, NER = 3, 2, 2, 5, 2
    J = inputs.couplings(L, S, seed=21)
    T = inputs.temperatures(0.4, 1.5, NT)

    def fresh():
        o = oracle.Oracle(L, S, NR, NT, NER, 4, 12, oracle.FP64, oracle.ACU, 1.0, 9)
        o.init(J, T)
        return o

    t_max = 24
    snaps = analysis.run_logged(OracleRunner(fresh()), t_max)
    res = analysis.analyse(snaps, t_max, T, NR)
    assert [(r.lo, r.hi) for r in res] == analysis.log2_bins(t_max)
    # the same chain, one EMCS at a time
    o = fresh()
    per_emcs, rts = [], [o.rt_count.copy()]
    for _ in range(t_max):
        ob = o.new_observables()
        o.run(1, ob)
        per_emcs.append(ob.acc.copy())
        rts.append(o.rt_count.copy())
    per_emcs = np.array(per_emcs)  # [t][S][NT][6]
    for r in res:
        block = per_emcs[r.lo - 1:r.hi].mean(axis=0)
        np.testing.assert_allclose(r.per_sample["e"], block[..., 0] / NR, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(r.per_sample["sdy"], block[..., 5], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(r.per_sample["ql"], block[..., 4], rtol=1e-12, atol=1e-14)
        np.testing.assert_array_equal(r.round_trips, (rts[r.hi] - rts[r.lo - 1]).astype(float))
        assert np.allclose(r.pq.sum(axis=1), 1.0)


def test_cluster_zoology_means():
    """Mean r-th largest cluster size per temperature over samples and pairs."""
    sizes = np.zeros((2, 2, 3, 2, 6), dtype=np.int32)
    sizes[0, 0, 1, 0, 0] = 10
    sizes[1, 1, 1, 0, 0] = 30
    sizes[:, :, 2, 1, 1] = 4
    z = analysis.cluster_zoology(sizes)
    assert z["majority_mean"].shape == (3, 6)
    assert z["majority_mean"][1, 0] == 10.0 and z["majority_mean"][0, 0] == 0.0
    assert z["minority_mean"][2, 1] == 4.0


def test_precision_statement_criteria_on_constructed_runs():
    """The FP32-vs-FP64 statement's arithmetic on runs whose answers are
    known: a constant energy offset shows up exactly as the mean paired
    difference, and a shifted overlap histogram fails the P(q) criterion while
    an identically distributed one passes it."""
    rng = np.random.default_rng(3)
    S, NT, B, n = 40, 3, 11, 4
    base = [rng.normal(-1.2, 0.05, (S, NT)) for _ in range(n)]
    noise = [rng.normal(0.0, 1e-5, (S, NT)) for _ in range(n)]
    p = np.exp(-0.5 * ((np.arange(B) - 5.0) / 2.0) ** 2)
    p /= p.sum()
    hists = [rng.multinomial(200000, p, size=NT).astype(float) for _ in range(2 * n)]
    fp64 = [analysis.FormRun(base[i], hists[i]) for i in range(n)]
    fp32 = [analysis.FormRun(base[i] + 3e-5 + noise[i], hists[n + i]) for i in range(n)]
    r = analysis.precision_statement(fp64, fp32)
    d = np.concatenate(noise, axis=0)
    assert np.allclose(r["e_diff_fp32_minus_fp64"], 3e-5 + d.mean(axis=0), atol=1e-15)
    assert np.allclose(r["e_diff_sigma"], d.std(axis=0, ddof=1) / np.sqrt(n * S))
    assert r["e_within_tolerance"] and not r["e_within_n_sigma"]
    assert r["e_temperatures_beyond_n_sigma"] == NT
    assert abs(r["e_z_bound_over_the_grid"] - 3.320) < 0.01  # 3 sigma over 3 temperatures
    assert abs(r["e_diff_averaged_over_T"] - (3e-5 + d.mean())) < 1e-15
    # one temperature: the grid bound is the plain 3 sigma
    one = [analysis.FormRun(f.e[:, :1], f.hist[:1]) for f in fp64]
    assert abs(analysis.precision_statement(one, [analysis.FormRun(f.e[:, :1], f.hist[:1]) for f in fp32])
               ["e_z_bound_over_the_grid"] - 3.0) < 1e-9
    assert r["pq_within_fp64_spread"]
    # the leave-one-out pools: run i of either form against the FP64 runs j != i
    pool0 = hists[1] + hists[2] + hists[3]
    assert np.allclose(r["pq_tv_mean_over_T"]["fp32"][0], analysis.total_variation(hists[n], pool0).mean())
    shifted = np.roll(p, 1) * 0.05 + p * 0.95
    bad = [analysis.FormRun(f.e, rng.multinomial(200000, shifted, size=NT).astype(float)) for f in fp32]
    assert not analysis.precision_statement(fp64, bad)["pq_within_fp64_spread"]
    tv = analysis.total_variation(np.array([[1.0, 3.0]]), np.array([[3.0, 1.0]]))
    assert np.allclose(tv, [0.5])
