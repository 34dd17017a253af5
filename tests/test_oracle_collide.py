"""Pins of the collision step: the claim rule by brute force, and the
CM-frame kinematics by conservation laws, an exact special case, an
independent Lorentz-boost check and isotropy."""
import itertools

import numpy as np
import pytest
from scipy import stats


def _pair_list(n):
    return [(a, b) for a in range(n) for b in range(a + 1, n)]


def _lex_first_maximal_matching(n, edges):
    """Brute force: among all maximal matchings of the candidate graph (edges
    given by their lexicographic pair index), the one whose sorted index
    list is lexicographically smallest."""
    pairs = _pair_list(n)
    best = None
    E = sorted(edges)
    for r in range(len(E) + 1):
        for sub in itertools.combinations(E, r):
            used = set()
            ok = True
            for k in sub:
                a, b = pairs[k]
                if a in used or b in used:
                    ok = False
                    break
                used |= {a, b}
            if not ok:
                continue
            # maximal: no remaining edge can be added
            if any(pairs[k][0] not in used and pairs[k][1] not in used
                   for k in E if k not in sub):
                continue
            cand = list(sub)
            if best is None or cand < best:
                best = cand
    return [pairs[k] for k in (best or [])]


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_claim_rule_is_lex_first_maximal_matching(orc, n):
    rng = np.random.default_rng(100 + n)
    kfac = 0.2
    pairs = _pair_list(n)
    for trial in range(60):
        p = rng.normal(size=(n, 3))
        E = np.linalg.norm(p, axis=1)
        edges = []
        u_acc = np.ones(len(pairs))          # u = 1 is never below P22 <= 2K < 1
        for k, (a, b) in enumerate(pairs):
            cos = p[a] @ p[b] / (E[a] * E[b])
            P = (1.0 - cos) * kfac            # v_rel = 1 - cos for massless
            if rng.random() < 0.5 and P > 1e-6:
                edges.append(k)
                u_acc[k] = 0.5 * P            # far below the threshold
        u_kin = rng.random(2 * len(pairs))
        newp, acc = orc.collide_cell_with_uniforms(p, kfac, u_acc, u_kin)
        assert acc == _lex_first_maximal_matching(n, edges), (n, trial)
        hit = {i for ab in acc for i in ab}
        for i in range(n):
            if i not in hit:                  # untouched members are bit-exact
                assert np.array_equal(newp[i], p[i])
        for a, b in acc:                      # each scattering conserves p
            assert np.allclose(newp[a] + newp[b], p[a] + p[b], rtol=0, atol=1e-13 * (E[a] + E[b]))


def _random_pairs(rng, m):
    """Momentum pairs covering soft, hard, boosted and nearly collinear ones."""
    out = []
    for i in range(m):
        pa = rng.normal(size=3) * np.exp(rng.uniform(-3, 3))
        kind = i % 4
        if kind == 0:
            pb = rng.normal(size=3) * np.exp(rng.uniform(-3, 3))
        elif kind == 1:     # nearly collinear, strongly boosted CM
            pb = pa * np.exp(rng.uniform(-2, 2)) + rng.normal(size=3) * 1e-5 * np.linalg.norm(pa)
        elif kind == 2:     # nearly back to back
            pb = -pa * np.exp(rng.uniform(-1, 1)) + rng.normal(size=3) * 1e-3
        else:               # very different energies
            pb = rng.normal(size=3) * 1e-4 * np.linalg.norm(pa)
        out.append((pa, pb))
    return out


def test_kinematics_conserves_energy_momentum_and_s(orc):
    rng = np.random.default_rng(3)
    worst_e = worst_p = worst_s = 0.0
    for pa, pb in _random_pairs(rng, 4000):
        uc, uphi = rng.random(2)
        qa, qb = orc.scatter_pair(pa, pb, uc, uphi)
        Ea, Eb = np.linalg.norm(pa), np.linalg.norm(pb)
        Et = Ea + Eb
        Ea2, Eb2 = np.linalg.norm(qa), np.linalg.norm(qb)
        worst_e = max(worst_e, abs((Ea2 + Eb2) - Et) / Et)
        worst_p = max(worst_p, np.max(np.abs((qa + qb) - (pa + pb))) / Et)
        # invariant mass: s = Et^2 - |P|^2 is the same before and after
        P = pa + pb
        s0 = 2 * Ea * Eb * (1 - (pa @ pb) / (Ea * Eb))
        s1 = 2 * Ea2 * Eb2 * (1 - (qa @ qb) / (Ea2 * Eb2))
        if s0 > 1e-6 * Et**2:
            worst_s = max(worst_s, abs(s1 - s0) / s0)
    assert worst_e <= 1e-12
    assert worst_p <= 1e-12
    assert worst_s <= 1e-9


def test_back_to_back_equal_energies_is_exact(orc):
    """P = 0 and Ea = Eb: the CM frame is the lab frame (gamma = 1 exactly),
    so the outgoing momenta are +-E n with n the drawn direction."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        E = float(np.exp(rng.uniform(-2, 2)))
        pa, pb = E * d, -E * d
        uc, uphi = rng.random(2)
        qa, qb = orc.scatter_pair(pa, pb, uc, uphi)
        Ecalc = np.linalg.norm(pa)
        cth = 2 * uc - 1
        sth = np.sqrt((1 - cth) * (1 + cth))
        n = np.array([sth * np.cos(2 * np.pi * uphi), sth * np.sin(2 * np.pi * uphi), cth])
        assert np.allclose(qa, Ecalc * n, rtol=0, atol=4e-16 * E)
        assert np.allclose(qb, -Ecalc * n, rtol=0, atol=4e-16 * E)


def _boost(E, p, beta):
    """General Lorentz boost of the four-vector (E, p) into the frame moving
    with velocity beta, via the 4x4 matrix (independent of the oracle)."""
    b2 = beta @ beta
    g = 1.0 / np.sqrt(1.0 - b2)
    L = np.eye(4)
    L[0, 0] = g
    L[0, 1:] = L[1:, 0] = -g * beta
    if b2 > 0:
        L[1:, 1:] += (g - 1) * np.outer(beta, beta) / b2
    v = L @ np.concatenate([[E], p])
    return v[0], v[1:]


def test_outgoing_direction_is_the_drawn_one_in_cm(orc):
    """Boosting the outgoing pair back into the CM frame gives back-to-back
    momenta E* (+n, -n), n the drawn direction, lower index along +n."""
    rng = np.random.default_rng(9)
    for _ in range(500):
        pa = rng.normal(size=3)
        pb = rng.normal(size=3) * 0.5
        uc, uphi = rng.random(2)
        qa, qb = orc.scatter_pair(pa, pb, uc, uphi)
        P = pa + pb
        Et = np.linalg.norm(pa) + np.linalg.norm(pb)
        beta = P / Et
        s = Et**2 - P @ P
        _, qa_cm = _boost(np.linalg.norm(qa), qa, beta)
        _, qb_cm = _boost(np.linalg.norm(qb), qb, beta)
        cth = 2 * uc - 1
        sth = np.sqrt(1 - cth**2)
        n = np.array([sth * np.cos(2 * np.pi * uphi), sth * np.sin(2 * np.pi * uphi), cth])
        assert np.allclose(qa_cm, 0.5 * np.sqrt(s) * n, atol=1e-10 * Et)
        assert np.allclose(qb_cm, -0.5 * np.sqrt(s) * n, atol=1e-10 * Et)


def test_cm_direction_is_isotropic(orc):
    """With Philox-like uniforms the CM polar cosine and azimuth of the
    outgoing particle are uniform (KS)."""
    rng = np.random.default_rng(11)
    pa = np.array([1.0, 0.2, -0.3])
    pb = np.array([-0.1, 0.8, 0.4])
    P = pa + pb
    Et = np.linalg.norm(pa) + np.linalg.norm(pb)
    beta = P / Et
    cths, phis = [], []
    for _ in range(3000):
        qa, _ = orc.scatter_pair(pa, pb, *rng.random(2))
        _, q = _boost(np.linalg.norm(qa), qa, beta)
        q = q / np.linalg.norm(q)
        cths.append(q[2])
        phis.append(np.arctan2(q[1], q[0]) % (2 * np.pi))
    assert stats.kstest(np.array(cths), stats.uniform(-1, 2).cdf).pvalue > 1e-3
    assert stats.kstest(np.array(phis), stats.uniform(0, 2 * np.pi).cdf).pvalue > 1e-3


def test_collinear_pair_left_unchanged(orc):
    pa = np.array([1.0, 2.0, 3.0])
    qa, qb = orc.scatter_pair(pa, 2.0 * pa, 0.3, 0.7)
    assert np.array_equal(qa, pa) and np.array_equal(qb, 2.0 * pa)
