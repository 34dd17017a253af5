"""Shared GPU-vs-oracle check of one step at full size (no GPU work here:
the caller passes GPU states fetched through the C ABI)."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def orc_params(orc, params):
    q = {k: v for k, v in params.items() if k not in ("step0", "cell_capacity")}
    return orc.make_params(**q)


def rows(a):
    a = np.asarray(a, dtype=np.int64).reshape(-1, 3)
    if len(a) == 0:
        return a
    return a[np.lexsort((a[:, 2], a[:, 1], a[:, 0]))]


def full_step_check(orc, got_prev, got, params, t, label, threads=16):
    """One traced oracle step from the GPU state got_prev at step index t
    must give the GPU state got, as the parity contract states it:
      * positions bit-exact for every particle;
      * the particles whose momenta the GPU step changed beyond free
        streaming (the same state stepped by the oracle with sigma = 0) are
        exactly the members of the oracle's claimed pairs;
      * momenta of every other particle bit-exact;
      * scattered momenta within 1e-12 (Ea + Eb) of the oracle's, with Ea + Eb
        the energy of the claimed pair they belong to.
    Returns the number of scattered particles."""
    n = len(got[0])
    say(f"[{label}] oracle: free streaming, {threads} threads")
    free = orc.State(*got_prev)
    orc.run(orc_params(orc, {**params, "sigma": 0.0}), free, t, 1, threads)
    say(f"[{label}] oracle: traced step")
    st = orc.State(*got_prev)
    tr = orc.step(orc_params(orc, params), st, t, trace=True)
    for d in range(3):
        assert np.array_equal(got[d], st[d]), f"{label}: positions differ on axis {d}"
        assert np.array_equal(free[d], st[d]), f"{label}: collisions moved a particle"
    claims = rows(tr["claim"])
    offs = tr["offsets"].astype(np.int64)
    ia = tr["perm"][offs[claims[:, 0]] + claims[:, 1]].astype(np.int64)
    ib = tr["perm"][offs[claims[:, 0]] + claims[:, 2]].astype(np.int64)
    claimed = np.zeros(n, bool)
    claimed[ia] = True
    claimed[ib] = True
    assert claimed.sum() == 2 * len(claims), f"{label}: a particle claimed twice"
    E = np.sqrt(free[3] ** 2 + free[4] ** 2 + free[5] ** 2)
    pair_e = np.zeros(n)
    pair_e[ia] = E[ia] + E[ib]
    pair_e[ib] = pair_e[ia]
    moved_g = np.zeros(n, bool)
    moved_o = np.zeros(n, bool)
    for d in range(3, 6):
        moved_g |= got[d] != free[d]
        moved_o |= st[d] != free[d]
    assert np.array_equal(moved_o, claimed), f"{label}: oracle moved != oracle claimed"
    assert np.array_equal(moved_g, claimed), (
        f"{label}: {int((moved_g & ~claimed).sum())} scattered on the GPU only, "
        f"{int((claimed & ~moved_g).sum())} claimed by the oracle only")
    for d in range(3, 6):
        assert np.array_equal(got[d][~claimed], st[d][~claimed]), f"{label}: unscattered p"
        dev = np.abs(got[d][claimed] - st[d][claimed])
        assert np.all(dev <= 1e-12 * pair_e[claimed]), (label, d, float(dev.max()))
    return int(claimed.sum())
