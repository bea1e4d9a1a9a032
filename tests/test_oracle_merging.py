"""Pins of the oracle's merging of superparticles (Sec. 2.3.2): two
superparticles of one species become one whose weight is the sum and whose
position and velocity are those of the centre of mass. Checked against what
that definition fixes independently of how the oracle writes it:

- the weight, the first moment sum w r and the momentum sum w v of every cell
  and species are unchanged;
- merging is a perfectly inelastic collision, so each merged pair loses the
  kinetic energy (1/2) m mu |v1 - v2|^2, mu = w1 w2 / (w1 + w2);
- a merged pair's position lies on the segment between its two positions,
  at the distance ratio w2 : w1 from them.

And the pair choice of the reading (per cell and species, ascending id order,
k = min(floor(N / 2), N - merge_max) leading pairs, the lower id kept, no pair
above w_max, nothing created in this step's collisions) by enumeration on
cells of known content.
"""
import numpy as np
import pytest

import oracle
from paper_2402_08404_amd import workloads as W


def _cell_load(cfg, counts, rng, wmax=9):
    """Particles in distinct cells, counts[c] of them in cell c, every
    species; ids are numbered in load order, so within a cell ids ascend in
    the order generated here."""
    pool = [(i, j, k) for k in range(4, cfg.nz - 4, 2) for j in range(1, cfg.ny - 2, 2)
            for i in range(1, cfg.nx - 2, 2)]
    cells = [pool[p] for p in rng.choice(len(pool), size=len(counts), replace=False)]
    load = {}
    for name in W.SPECIES:
        X = np.concatenate([np.full(n, c[0]) + rng.uniform(0.01, 0.99, n) for c, n in zip(cells, counts)])
        Y = np.concatenate([np.full(n, c[1]) + rng.uniform(0.01, 0.99, n) for c, n in zip(cells, counts)])
        Z = np.concatenate([np.full(n, c[2]) + rng.uniform(0.01, 0.99, n) for c, n in zip(cells, counts)])
        m = len(X)
        load[name] = {"x": X, "y": Y, "z": Z, "vx": rng.normal(0, 0.01, m), "vy": rng.normal(0, 0.01, m),
                      "vz": rng.normal(0, 0.01, m), "w": rng.integers(1, wmax + 1, m)}
    return load, cells


def _cell_of(d):
    return np.floor(d["x"]).astype(int) * 10 ** 8 + np.floor(d["y"]).astype(int) * 10 ** 4 + \
        np.floor(d["z"]).astype(int)


def _sums(d):
    c = _cell_of(d)
    out = {}
    for cc in np.unique(c):
        m = c == cc
        w = d["w"][m].astype(float)
        out[int(cc)] = (int(d["w"][m].sum()),) + tuple(float((w * d[k][m]).sum()) for k in
                                                      ("x", "y", "z", "vx", "vy", "vz"))
    return out


def pin_merge_conservation():
    cfg = W.small(nx=24, ny=24, nz=24, tip_r=1e-9, tip_h=2e-9)
    cfg.merge_max, cfg.w_max = 2, 1000
    rng = np.random.default_rng(81)
    load, _ = _cell_load(cfg, rng.integers(1, 12, 150), rng)
    o = oracle.Oracle(cfg, laplace=False)
    o.load(load)
    before = o.state()
    n = o.merge(o.next_id)
    after = o.state()
    assert n > 300
    for s in range(3):
        b, a = _sums(before[s]), _sums(after[s])
        assert b.keys() == a.keys()
        for c in b:
            assert b[c][0] == a[c][0]
            np.testing.assert_allclose(a[c][1:], b[c][1:], rtol=1e-13, atol=1e-15)
        # energy: each merged pair loses (1/2) m mu |v1 - v2|^2 (per unit mass,
        # in grid units)
        bi = {int(i): k for k, i in enumerate(before[s]["id"])}
        ai = {int(i): k for k, i in enumerate(after[s]["id"])}
        gone = sorted(set(bi) - set(ai))
        loss = 0.0
        for g in gone:
            # the partner is the surviving id just below in the same cell
            # (pairs are consecutive in id order)
            kb = bi[g]
            cell = _cell_of({k: before[s][k][kb:kb + 1] for k in ("x", "y", "z")})[0]
            same = [int(i) for i in before[s]["id"] if int(i) < g and int(i) in ai and
                    _cell_of({k: before[s][k][bi[int(i)]:bi[int(i)] + 1] for k in ("x", "y", "z")})[0] == cell]
            p = max(same)
            kp = bi[p]
            w1, w2 = float(before[s]["w"][kp]), float(before[s]["w"][kb])
            mu = w1 * w2 / (w1 + w2)
            dv = np.array([before[s][k][kp] - before[s][k][kb] for k in ("vx", "vy", "vz")])
            loss += 0.5 * mu * float(dv @ dv)
            # the merged position divides the segment in the ratio w2 : w1
            ka = ai[p]
            ra = np.array([before[s][k][kp] for k in ("x", "y", "z")])
            rb = np.array([before[s][k][kb] for k in ("x", "y", "z")])
            rm = np.array([after[s][k][ka] for k in ("x", "y", "z")])
            assert after[s]["w"][ka] == w1 + w2
            np.testing.assert_allclose(np.linalg.norm(rm - ra) * w1, np.linalg.norm(rm - rb) * w2, rtol=1e-9)
            np.testing.assert_allclose(np.linalg.norm(rm - ra) + np.linalg.norm(rm - rb), np.linalg.norm(ra - rb),
                                       rtol=1e-12)

        def ke(d):
            return 0.5 * float((d["w"] * (d["vx"] ** 2 + d["vy"] ** 2 + d["vz"] ** 2)).sum())

        assert ke(before[s]) - ke(after[s]) == pytest.approx(loss, rel=1e-9)


def test_merge_conserves_weight_centre_and_momentum():
    pin_merge_conservation()


def test_merge_pair_choice():
    """Cells with N = 1 .. 12 superparticles of every species and merge_max = 4:
    k = min(floor(N / 2), N - 4) pairs merge, the survivors are the ids of
    rank 0, 2, .., 2k - 2 and all ids of rank 2k and above."""
    pin_pair_choice()


def pin_pair_choice():
    cfg = W.small(nx=24, ny=24, nz=24, tip_r=1e-9, tip_h=2e-9)
    cfg.merge_max, cfg.w_max = 4, 1000
    rng = np.random.default_rng(82)
    counts = list(range(1, 13)) * 3
    load, cells = _cell_load(cfg, counts, rng)
    o = oracle.Oracle(cfg, laplace=False)
    o.load(load)
    o.merge(o.next_id)
    st = o.state()
    base = 0
    for s in range(3):
        alive = set(int(i) for i in st[s]["id"])
        want = set()
        for N in counts:
            ids = list(range(base, base + N))
            k = min(N // 2, N - 4) if N > 4 else 0
            want |= {ids[2 * q] for q in range(k)} | set(ids[2 * k:])
            base += N
        assert alive == want
        assert o.merges[s] == sum(min(N // 2, N - 4) for N in counts if N > 4)


def test_merge_respects_w_max_and_id_limit():
    """A pair whose summed weight exceeds w_max is kept apart, and
    superparticles with ids at or above the limit take no part."""
    pin_w_max_and_id_limit()


def pin_w_max_and_id_limit():
    cfg = W.small(nx=24, ny=24, nz=24, tip_r=1e-9, tip_h=2e-9)
    cfg.merge_max, cfg.w_max = 1, 10
    rng = np.random.default_rng(83)
    load, _ = _cell_load(cfg, [2] * 40, rng, wmax=8)
    o = oracle.Oracle(cfg, laplace=False)
    o.load(load)
    w = [o.state()[s]["w"].reshape(-1, 2).sum(axis=1) for s in range(3)]
    limit = o.next_id - 2 * 20          # the neutrals' last 20 cells are not candidates
    o.merge(limit)
    for s in range(3):
        ok = w[s] <= 10
        if s == 2:
            ok[20:] = False
        assert o.merges[s] == int(ok.sum())
        assert len(o.state()[s]["id"]) == 80 - int(ok.sum())


def test_merge_in_whole_steps_keeps_charge_and_units():
    """Whole weighted steps of the tiny workload with merging every step
    (merge_max 1): every species merges, and the deposited charge equals the
    charge of the superparticles after merging."""
    cfg = W.tiny()
    cfg.merge_every, cfg.merge_max, cfg.w_max = 1, 1, 64
    rng = np.random.default_rng(84)
    load = W.initial_load(cfg)
    for name in load:
        load[name]["w"] = rng.integers(1, 4, len(load[name]["x"]))
    o = oracle.Oracle(cfg)
    o.load(load)
    o.deposit()
    o.solve(rtol=1e-8)
    for _ in range(3):
        o.step(rtol=1e-8)
        st = o.state()
        assert int(o.Q.sum()) == 2 ** 40 * (int(st[1]["w"].sum()) - int(st[0]["w"].sum()))
    m = o.moments()
    assert (m["merges"] > 0).all()
