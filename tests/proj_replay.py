"""Replay of a projection sequence through the library and the oracle side by side.

Both sides receive the same (b_n, x_n) pairs (the replay protocol: two
independent solve loops differ at the solve tolerance, so their guesses could
not be compared), and after every update the accept / reject decisions are
compared.  Where they differ and the oracle's ratio nu / nu0 lies within a
relative 1e-6 of eps_rel -- a decision that rounding can flip -- the oracle's
update is redone with the library's decision forced (the basis after a flip
is not unique, so the comparison could not go on otherwise); anywhere else a
differing decision fails the replay.

Guess tolerance for FP64 storage: relative max(1e-12, 1e-14 a), a = max
nu0 / nu of the stored columns (the normalisation of a column accepted with
ratio nu / nu0 amplifies its rounding by nu0 / nu, so two correct FP64
implementations that sum in different orders agree only to about u a).
"""
import copy

import numpy as np

from gpu_helpers import dev, host, rel_inf

AMBIGUOUS = 1e-6   # relative distance of nu / nu0 from eps_rel within which a decision may flip


def guess_tol(amp):
    return max(1e-12, 1e-14 * amp)


def _fetch_raw(L, g, N, d):
    import torch

    out = []
    buf = torch.empty(N, dtype=torch.float64, device="cuda")
    for j in range(d):
        sx = L.guess_history_raw(g, 0, j, buf)
        xs = host(buf).copy()
        sb = L.guess_history_raw(g, 1, j, buf)
        bs = host(buf).copy()
        assert sx == sb
        out.append((xs, bs, sx))
    return out


def resync(L, g, ref, raw):
    """Give the oracle the library's stored history (values, scales, factor R): the next
    update then starts from identical states on both sides."""
    ref.S = [xs.copy() for xs, _, _ in raw]
    ref.T = [bs.copy() for _, bs, _ in raw]
    ref.sig = [sc for _, _, sc in raw]
    ref.mu = [sc * max(float(np.max(np.abs(xs))), float(np.max(np.abs(bs)))) for xs, bs, sc in raw]
    ref.R = L.guess_proj_factor(g)


def replay(L, g, ref, B, X, eps, Aop=None, use_ax=False, raw=False, factors=False, sync=False):
    """Run the sequence through context g and oracle ref; returns one row per step.

    Each row: got / want guesses, the amplification before and after the step, decisions, d, the
    oracle's ratio, whether the decision was forced, the library's info, the largest magnitude
    of the step's raw pair (x, A x), and optionally the library's raw stored columns with the
    oracle's (S, T, sigma) and both factors R.  With `sync` the oracle takes the library's
    stored history after every step (so each step is compared from identical states)."""
    import torch

    N = len(B[0])
    x0 = torch.empty(N, dtype=torch.float64, device="cuda")
    rows = []
    for b, x in zip(B, X):
        L.guess_form(g, dev(b), x0)
        want = ref.form(b)
        amp = ref.amplification
        got = host(x0)
        Ax = Aop(x) if use_ax else None
        L.guess_update(g, dev(x), None if Ax is None else dev(Ax))
        info = L.guess_get_info(g)
        acc = bool(info["last_accepted"])
        saved = copy.deepcopy(ref)
        acc_ref = ref.update(x, Ax)
        ratio = ref.last_nu / ref.last_nu0 if ref.last_nu0 else 0.0
        forced = False
        if acc != acc_ref and abs(ratio - eps) <= AMBIGUOUS * eps:
            ref = saved
            acc_ref = ref.update(x, Ax, decide=acc)
            forced = True
        ax = Ax if Ax is not None else (Aop(x) if Aop is not None else x)
        row = dict(got=got, want=want, amp=amp, amp_after=ref.amplification, acc=acc, acc_ref=acc_ref,
                   d=info["count"], d_ref=ref.d, ratio=ratio, forced=forced, info=info,
                   xmax=max(float(np.max(np.abs(x))), float(np.max(np.abs(ax)))))
        if raw or sync:
            row["raw"] = _fetch_raw(L, g, N, info["count"])
            row["ref_cols"] = [(S.copy(), T.copy(), sg) for S, T, sg in zip(ref.S, ref.T, ref.sig)]
        if factors:
            row["R"], row["R_ref"] = L.guess_proj_factor(g), ref.R.copy()
        rows.append(row)
        if sync and row["d"] == row["d_ref"]:
            resync(L, g, ref, row["raw"])
    return rows, ref


def check_rows(rows, strict=False, label=""):
    """Every step: decisions agree (after forcing), d agrees, and the guess is within the
    FP64 tolerance.  Returns the number of steps checked (all of them) and prints the largest
    error in units of u a (u = 2^-53)."""
    worst = 0.0
    for q, r in enumerate(rows):
        assert r["acc"] == r["acc_ref"], f"{label}: decision differs at step {q} (ratio {r['ratio']!r})"
        assert r["d"] == r["d_ref"], (label, q, r["d"], r["d_ref"])
        if np.max(np.abs(r["want"])) == 0:
            assert not r["got"].any(), (label, q)
            continue
        tol = 1e-12 if strict else guess_tol(r["amp"])
        err = rel_inf(r["got"], r["want"])
        worst = max(worst, err / (2.0 ** -53 * max(1.0, r["amp"])))
        assert err <= tol, (label, q, err, r["amp"])
    forced = sum(r["forced"] for r in rows)
    print(f"[replay] {label}: {len(rows)} steps, {forced} forced decisions, max error {worst:.1f} u a",
          flush=True)
    return len(rows)
