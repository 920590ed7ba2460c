"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test fixes the oracle to something independent of its own code: values
derived by hand from the paper's definitions (``tests/golden``), closed forms,
exact rational brute force, 50-digit brute force, invariances, and a
black-box library cross-check.  Between them they catch a dropped term, a
wrong sign or factor, a transposed index or a wrong tie/merge rule anywhere in
the oracle.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "hand_cases.json")))


# --------------------------------------------------------------------------
# Hand-derived worked examples
# --------------------------------------------------------------------------

def test_flat_window_inclusive(orc):
    """eq. (12)-(13): the window includes the point at exactly distance h."""
    g = GOLD["flat_window"]
    X = np.array(g["points"], np.float32)
    m1, w1 = orc.mean(X, g["seed"], g["h"], "flat")
    assert w1 == 4.0
    assert m1.tolist() == g["step1"]
    S, st, it, sh = orc.step(X, [g["seed"]], g["h"], "flat", tol=1e-3, n_iter=10)
    assert S[0].tolist() == g["step2"]
    assert it[0] == g["converged_at"] and st[0] == orc.CONVERGED and sh[0] == 0.0


def test_gaussian_two_point_closed_form(orc):
    g = GOLD["gaussian_two_point"]
    X = np.array(g["points"], np.float32)
    m1, _ = orc.mean(X, g["seed"], g["h"], "gaussian")
    assert abs(m1[0] - g["step1"][0]) <= 1e-15 and m1[1] == 0.0
    # general two-point form m = x1 + (x2 - x1) w / (1 + w), w = exp(-a^2/(2h^2))
    for a, h in [(0.5, 1.0), (3.0, 2.0), (1.0, 0.25)]:
        X = np.array([[1.0, -2.0], [1.0 + a, -2.0]], np.float32)
        w = math.exp(-a * a / (2 * h * h))
        m, _ = orc.mean(X, X[0].astype(np.float64), h, "gaussian")
        assert abs(m[0] - (1.0 + a * w / (1 + w))) < 1e-14 and m[1] == -2.0


def test_greedy_merge_and_tie_label(orc):
    g = GOLD["greedy_merge_line"]
    X = np.array(g["points"], np.float32)
    r = orc.fit(X, g["h"], kernel="flat", all_points=True,
                merge_radius=g["merge_radius"])
    assert r.status == 0
    assert r.drawn_final.tolist() == g["finals"]
    assert r.drawn_iters.tolist() == g["iters"]
    assert r.modes.tolist() == g["modes"]
    assert r.counts.tolist() == g["counts"]
    assert r.labels.tolist() == g["labels"]
    assert r.margin.tolist() == g["margins"]


def test_splitmix64_published_outputs(orc):
    g = GOLD["splitmix64_seed0"]
    assert [f"{v:016x}" for v in orc.splitmix64_stream(0, 3)] == g["outputs_hex"]


def test_merge_joins_first_of_two_modes(orc):
    g = GOLD["merge_first_of_two"]
    X = np.array(g["points"], np.float32)
    r = orc.fit(X, g["h"], kernel="flat", all_points=True, merge_radius=g["merge_radius"])
    assert r.modes.tolist() == g["modes"] and r.counts.tolist() == g["counts"]
    assert r.labels.tolist() == g["labels"]


def test_fisher_yates_hand_slots(orc):
    g = GOLD["fisher_yates_first_five"]
    d, _ = orc.draw(g["rng_seed"], np.arange(100, dtype=np.int32), 5)
    assert d.tolist() == g["draw"]


def _isolated_points(n, h):
    # a grid with spacing 2h: no two points share a window
    side = int(math.ceil(math.sqrt(n)))
    ij = np.array([(i, j) for i in range(side) for j in range(side)][:n], np.float32)
    return ij * np.float32(2.0 * h)


def test_seed_count_doubling(orc):
    g = GOLD["seed_count_doubling"]
    X = _isolated_points(2000, 1.0)
    r = orc.fit(X, 1.0, kernel="flat")
    assert r.round_N.tolist() == g["round_N"]
    assert r.round_B.tolist() == g["round_B"]
    assert r.round_M.tolist() == g["round_M"]
    assert r.k == 2000 and sorted(r.drawn.tolist()) == list(range(2000))


def test_seed_count_stops_at_L_times_M(orc):
    """Section II-D: the loop ends once N >= L*M even with a non-empty pool."""
    rng = np.random.default_rng(3)
    # 10 tight clusters far apart: M = 10 after round 1, 128 >= 80 -> one round
    C = np.arange(10)[:, None] * np.array([[100.0, 0.0]])
    X = (C[np.repeat(np.arange(10), 300)] + 0.05 * rng.standard_normal((3000, 2))).astype(np.float32)
    r = orc.fit(X, 1.0, kernel="flat", cover_radius=0.0)
    assert r.round_N.tolist() == [128] and r.k == 10
    # with L = 16: 128 < 160, so a second round of 256 runs; then 256 >= 160
    r = orc.fit(X, 1.0, kernel="flat", cover_radius=0.0, L=16)
    assert r.round_N.tolist() == [128, 256] and r.k == 10
    # equality ends the loop: 16 clusters, N = 128 = 8 * 16
    C = np.arange(16)[:, None] * np.array([[100.0, 0.0]])
    X = (C[np.repeat(np.arange(16), 300)] + 0.05 * rng.standard_normal((4800, 2))).astype(np.float32)
    r = orc.fit(X, 1.0, kernel="flat", cover_radius=0.0)
    assert r.k == 16 and r.round_N.tolist() == [128]


# --------------------------------------------------------------------------
# Seed pool, coverage and early stopping
# --------------------------------------------------------------------------

def test_coverage_removes_points_within_radius(orc):
    """A tight blob (all points within h of its mode) plus isolated points:
    after round 1 no later round may draw a blob point or a drawn point."""
    rng = np.random.default_rng(5)
    blob = 0.1 * rng.standard_normal((1000, 2))
    iso = _isolated_points(1000, 1.0) + np.float32(50.0)
    X = np.concatenate([blob, iso]).astype(np.float32)
    r = orc.fit(X, 1.0, kernel="flat")
    rounds = r.rounds()
    assert len(rounds) >= 2
    assert (rounds[0] < 1000).any()            # the blob was hit in round 1
    seen = set(rounds[0].tolist())
    for later in rounds[1:]:
        assert (later >= 1000).all()           # blob points were covered
        assert not (set(later.tolist()) & seen)
        seen |= set(later.tolist())
    # every isolated point that was drawn is its own mode; the blob is one mode
    assert r.k == 1 + int((r.drawn >= 1000).sum())


def test_gamma_early_stop(orc):
    """Section II-C: the batch stops once ceil(gamma*B) seeds converged and
    discards the rest.  Isolated seeds converge at the first update (shift 0);
    seeds on a two-point Gaussian pair need many updates."""
    pairs = [[100.0 * i, 0.0] for i in range(4)] + [[100.0 * i + 1.0, 0.0] for i in range(4)]
    iso = [[0.0, 100.0 + 100.0 * i] for i in range(4)]
    X = np.array(pairs + iso, np.float32)
    # 12 seeds, gamma = 1/4: need = 3 <= 4 -> stops after iteration 1, the 8
    # pair seeds are discarded unconverged
    r = orc.fit(X, 1.0, kernel="gaussian", all_points=True, gamma=0.25)
    assert r.round_T.tolist() == [1]
    assert r.drawn_status.tolist() == [0] * 8 + [1] * 4
    assert r.k == 4 and r.pairs == 12 * 12
    # gamma = 5/12 needs 5 converged seeds: the batch runs on until two pair
    # seeds have converged too (they all converge at the same update)
    r = orc.fit(X, 1.0, kernel="gaussian", all_points=True, gamma=5.0 / 12.0)
    T = r.round_T[0]
    assert T > 1 and (r.drawn_status == 1).all() and (r.drawn_iters[:8] == T).all()
    # gamma = 1: everything converges
    r = orc.fit(X, 1.0, kernel="gaussian", all_points=True, gamma=1.0)
    assert (r.drawn_status == 1).all() and r.round_T[0] > 1
    assert r.k == 8


def test_max_iter_discards(orc):
    X = np.array([[0.0, 0.0], [1.0, 0.0]], np.float32)
    r = orc.fit(X, 1.0, kernel="gaussian", all_points=True, max_iter=1)
    assert r.status == -4 and r.k == 0 and (r.drawn_status == 0).all()


# --------------------------------------------------------------------------
# Closed forms
# --------------------------------------------------------------------------

def test_single_point_is_its_own_mean(orc):
    X = np.array([[3.25, -1.5, 7.0]], np.float32)
    for s in ([0.0, 0.0, 0.0], [3.0, -1.0, 7.5]):
        m, w = orc.mean(X, s, 2.0, "gaussian")
        # (w x) / w: two roundings, so at most 2 ulp from x
        x = X[0].astype(np.float64)
        assert (np.abs(m - x) <= 2 * np.spacing(np.abs(x))).all() and w > 0


def test_flat_small_diameter_set(orc):
    """Diameter <= h: one update reaches the sample mean, the next shifts 0;
    one mode, every label 0."""
    rng = np.random.default_rng(1)
    X = rng.uniform(0, 0.5, (37, 3)).astype(np.float32)   # diameter < 0.87
    mean = X.astype(np.float64).mean(0)
    S, st, it, sh = orc.step(X, X[:5].astype(np.float64), 1.0, "flat", n_iter=10)
    assert np.abs(S - mean).max() < 1e-15 and (it == 2).all() and (st == 1).all()
    r = orc.fit(X, 1.0, kernel="flat", all_points=True)
    assert r.k == 1 and (r.labels == 0).all()


def test_symmetric_set_fixed_point(orc):
    """Pairs x, 2 mu - x: mu is an exact fixed point of the update."""
    rng = np.random.default_rng(2)
    mu = np.array([4.0, -2.0], np.float64)
    half = rng.integers(-1024, 1025, (50, 2)) / 1024.0   # exact in float32
    X = np.concatenate([mu + half, mu - half]).astype(np.float32)
    assert np.array_equal(X[:50].astype(np.float64) - mu, mu - X[50:].astype(np.float64))
    for h in (0.5, 1.0, 3.0):
        m, _ = orc.mean(X, mu, h, "gaussian")
        assert np.abs(m - mu).max() <= 1e-14
        m, _ = orc.mean(X, mu, h, "flat")
        assert np.abs(m - mu).max() <= 1e-14


def test_gaussian_blob_contraction(orc):
    """Population identity for a Gaussian blob N(mu, s^2 I) under the Gaussian
    kernel: m(s) - mu = J (s - mu), J = s^2/(s^2 + h^2).  With exp(-q/h^2)
    instead of exp(-q/(2h^2)) J would be 0.24 instead of 0.138."""
    rng = np.random.default_rng(4)
    sig, h = 2.0, 5.0
    mu = np.array([10.0, 20.0])
    X = (mu + sig * rng.standard_normal((400_000, 2))).astype(np.float32)
    J = sig ** 2 / (sig ** 2 + h ** 2)
    emp_mu = X.astype(np.float64).mean(0)
    for off in ([3.0, 0.0], [0.0, -4.0], [2.0, 2.0]):
        s = mu + np.array(off)
        m, _ = orc.mean(X, s, h, "gaussian")
        ratio = np.dot(m - emp_mu, s - emp_mu) / np.dot(s - emp_mu, s - emp_mu)
        assert abs(ratio - J) < 0.01, (ratio, J)


def test_well_separated_blobs_give_k_clusters(orc):
    rng = np.random.default_rng(6)
    k, h, sig = 7, 1.0, 0.2
    C = rng.permutation(k)[:, None] * np.array([[0.0, 40.0, 0.0]]) + np.array([5.0, 0.0, -3.0])
    y = np.repeat(np.arange(k), 200)
    X = (C[y] + sig * rng.standard_normal((y.size, 3))).astype(np.float32)
    for all_points in (True, False):
        for kern in ("gaussian", "flat"):
            r = orc.fit(X, h, kernel=kern, all_points=all_points)
            assert r.status == 0 and r.k == k
            # labels equal the generating ids up to a permutation
            pairs = set(zip(y.tolist(), r.labels.tolist()))
            assert len(pairs) == k
            # each mode lies near its blob centre
            for j in range(k):
                c = C[y[r.labels == j][0]]
                assert np.linalg.norm(r.modes[j] - c) < 4 * sig / math.sqrt(200) + 0.05


# --------------------------------------------------------------------------
# Exact brute force
# --------------------------------------------------------------------------

def _frac_trajectory(P, s, h2, tol_h2, max_iter=100):
    """Exact rational iteration of the flat-window mean (eq. 12-15)."""
    traj = []
    for _ in range(max_iter):
        win = [p for p in P if sum((a - b) ** 2 for a, b in zip(p, s)) <= h2]
        if any(sum((a - b) ** 2 for a, b in zip(p, s)) == h2 for p in P) and traj:
            return None   # an exact boundary hit after rounding: not comparable
        c = len(win)
        nxt = tuple(sum(p[k] for p in win) / c for k in range(len(s)))
        d2 = sum((a - b) ** 2 for a, b in zip(nxt, s))
        traj.append(nxt)
        s = nxt
        if d2 < tol_h2:
            break
    return traj


def test_flat_exact_rational_bruteforce(orc):
    rng = np.random.default_rng(7)
    h, tol = 3.0, 1e-3
    h2 = Fraction(9)
    tol_h2 = Fraction(float(np.float32(tol))) ** 2 * h2
    checked = 0
    for case in range(40):
        n = int(rng.integers(2, 25))
        P = rng.integers(0, 9, (n, 2))
        X = P.astype(np.float32)
        Pf = [tuple(Fraction(int(v)) for v in p) for p in P]
        for j in range(min(n, 6)):
            traj = _frac_trajectory(Pf, Pf[j], h2, tol_h2)
            if traj is None:
                continue
            S, st, it, _ = orc.step(X, X[j:j + 1].astype(np.float64), h, "flat",
                                    tol=tol, n_iter=100)
            assert it[0] == len(traj) and st[0] == 1
            exact = [float(v) for v in traj[-1]]
            assert np.abs(S[0] - exact).max() <= 4 * np.spacing(np.abs(exact).max() + 1)
            # the first update is exact up to one rounding of each quotient
            m1, _ = orc.mean(X, X[j].astype(np.float64), h, "flat")
            assert m1.tolist() == [float(v) for v in traj[0]]
            checked += 1
    assert checked > 100


def test_gaussian_mpmath_bruteforce(orc):
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    rng = np.random.default_rng(8)
    for case in range(10):
        n, d = int(rng.integers(1, 64)), int(rng.integers(1, 6))
        X = (3.0 * rng.standard_normal((n, d))).astype(np.float32)
        s = rng.standard_normal(d) * 2.0
        h = float(rng.uniform(0.5, 4.0))
        num = [mp.mpf(0)] * d
        den = mp.mpf(0)
        for x in X.astype(np.float64):
            q = sum((mp.mpf(float(a)) - mp.mpf(float(b))) ** 2 for a, b in zip(x, s))
            w = mp.exp(-q / (2 * mp.mpf(h) ** 2))
            den += w
            num = [u + w * mp.mpf(float(a)) for u, a in zip(num, x)]
        exact = np.array([float(u / den) for u in num])
        m, W = orc.mean(X, s, h, "gaussian")
        assert np.abs(m - exact).max() <= 1e-13 * (1 + np.abs(exact).max())
        assert abs(W - float(den)) <= 1e-13 * float(den)


# --------------------------------------------------------------------------
# Invariances
# --------------------------------------------------------------------------

def _blobs(seed, n=600, d=2):
    rng = np.random.default_rng(seed)
    C = rng.uniform(0, 60, (4, d))
    y = rng.integers(0, 4, n)
    X = C[y] + 1.5 * rng.standard_normal((n, d))
    # on a 2^-10 grid, so power-of-two shifts and scalings stay exact in float32
    return (np.round(X * 1024.0) / 1024.0).astype(np.float32)


def test_translation_invariance(orc):
    X = _blobs(10)
    t = np.array([1024.0, -512.0], np.float32)   # power-of-two shift: exact in float32
    a = orc.fit(X, 4.0, all_points=True)
    b = orc.fit(X + t, 4.0, all_points=True)
    assert np.array_equal((X + t).astype(np.float64), X.astype(np.float64) + t)
    assert a.k == b.k and (a.labels == b.labels).all()
    assert np.abs(a.modes + t - b.modes).max() < 1e-8


def test_rotation_invariance(orc):
    X = _blobs(11)
    th = 0.6
    Q = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    a = orc.fit(X, 4.0, all_points=True)
    Xr = (X.astype(np.float64) @ Q.T).astype(np.float32)
    b = orc.fit(Xr, 4.0, all_points=True)
    assert a.k == b.k
    # float32 rounding of the rotated input perturbs modes by ~1e-6
    assert np.abs(a.modes @ Q.T - b.modes).max() < 1e-4
    assert (a.labels == b.labels).mean() > 0.999


def test_scaling_invariance(orc):
    X = _blobs(12)
    a = orc.fit(X, 4.0, all_points=True)
    b = orc.fit(X * np.float32(8.0), 32.0, all_points=True)  # exact power-of-two scale
    assert a.k == b.k and (a.labels == b.labels).all()
    assert np.abs(a.modes * 8.0 - b.modes).max() < 1e-9


def test_permutation_invariance(orc):
    X = _blobs(13)
    perm = np.random.default_rng(0).permutation(X.shape[0])
    a = orc.fit(X, 4.0, all_points=True)
    b = orc.fit(X[perm], 4.0, all_points=True)
    assert a.k == b.k
    # modes are the same set up to order and tol-level representative changes
    for m in a.modes:
        assert np.min(np.linalg.norm(b.modes - m, axis=1)) < 1e-2
    # the partition is the same
    la, lb = a.labels[perm], b.labels
    assert len(set(zip(la.tolist(), lb.tolist()))) == a.k


def test_fixed_point_of_a_mode(orc):
    X = _blobs(14)
    h, tol = 4.0, 1e-3
    r = orc.fit(X, h, all_points=True, tol=tol)
    S, st, it, sh = orc.step(X, r.modes, h, n_iter=1, tol=tol)
    # one more update from a converged mode moves it less than tol*h/(1-J)
    J = 1.5 ** 2 / (1.5 ** 2 + h ** 2)
    assert np.sqrt(sh).max() < tol * h / (1 - J)


def test_thread_count_does_not_change_results(orc):
    X = _blobs(15, n=1500)
    a = orc.fit(X, 4.0, nthreads=1)
    b = orc.fit(X, 4.0, nthreads=8)
    assert a.k == b.k and np.array_equal(a.modes, b.modes)
    assert np.array_equal(a.labels, b.labels) and np.array_equal(a.drawn, b.drawn)


# --------------------------------------------------------------------------
# Seed selection primitives
# --------------------------------------------------------------------------

def test_partial_fisher_yates_is_a_uniform_draw(orc):
    pool = np.arange(100, 140, dtype=np.int32)
    d, _ = orc.draw(123, pool, 40)
    assert sorted(d.tolist()) == pool.tolist()        # full shuffle is a permutation
    d, _ = orc.draw(123, pool, 10)
    assert len(set(d.tolist())) == 10 and set(d.tolist()) <= set(pool.tolist())
    # first slot is uniform over the pool (chi-square over many seeds)
    counts = np.zeros(8, int)
    for s in range(4000):
        counts[orc.draw(s, np.arange(8, dtype=np.int32), 1)[0][0]] += 1
    chi2 = ((counts - 500) ** 2 / 500).sum()
    assert chi2 < 24.3      # 7 dof, p = 0.001


# --------------------------------------------------------------------------
# Black-box cross-check
# --------------------------------------------------------------------------

def test_sklearn_blackbox_flat_all_points(orc):
    sk = pytest.importorskip("sklearn.cluster")
    rng = np.random.default_rng(9)
    C = np.array([[0.0, 0.0], [30.0, 5.0], [10.0, 40.0], [-25.0, 20.0]])
    y = np.repeat(np.arange(4), 150)
    X = (C[y] + 1.0 * rng.standard_normal((600, 2))).astype(np.float32)
    h = 4.0
    r = orc.fit(X, h, kernel="flat", all_points=True)
    ms = sk.MeanShift(bandwidth=h, bin_seeding=False, cluster_all=True).fit(X.astype(np.float64))
    assert r.k == len(ms.cluster_centers_)
    assert len(set(zip(r.labels.tolist(), ms.labels_.tolist()))) == r.k
    for c in ms.cluster_centers_:
        assert np.min(np.linalg.norm(r.modes - c, axis=1)) < 0.05
