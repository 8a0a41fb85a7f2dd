"""Helpers shared by the GPU parity tests (host <-> device copies, comparisons)."""
import sys

import numpy as np


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def announce(msg):
    """Name the case on stdout before a GPU step (flushed)."""
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def rel_inf(a, b):
    """max |a - b| / max(max |b|, tiny)."""
    a, b = np.asarray(a), np.asarray(b)
    scale = max(float(np.max(np.abs(b))) if b.size else 0.0, 1e-300)
    return float(np.max(np.abs(a - b))) / scale if a.size else 0.0


def assert_within(got, want, bound, hist=None, label=""):
    """Elementwise |got - want| <= bound; on failure report the worst elements."""
    got, want, bound = np.asarray(got), np.asarray(want), np.asarray(bound)
    bad = np.nonzero(~(np.abs(got - want) <= bound))[0]
    if bad.size:
        lines = [f"{label}: {bad.size} elements outside the bound"]
        for i in bad[:5]:
            h = "" if hist is None else " hist=" + repr([float(v[i]) for v in hist])
            lines.append(f"  i={i} got={got[i]!r} want={want[i]!r} bound={bound[i]!r}{h}")
        raise AssertionError("\n".join(lines))
