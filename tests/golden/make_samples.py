"""Write sampled FP64 oracle values for the full-size workloads.

Calls only ``oracle`` and ``workloads`` (never the GPU library), so every
stored number is the oracle's.  Output: tests/golden/<name>_samples.npz with
the canonical mu jet, response traces, max |P^(k)| and the values of P0,
P1[d], P2[d] at a fixed set of seeded (i, j) positions (random pairs plus
diagonal entries).

    python tests/golden/make_samples.py banded8192 cubic2048
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402


def sample_positions(n, seed=12345, pairs=1024, diag=1024):
    rng = np.random.default_rng(seed)
    i = rng.integers(0, n, pairs)
    j = rng.integers(0, n, pairs)
    k = rng.choice(n, size=min(diag, n), replace=False)
    return np.concatenate([i, k]), np.concatenate([j, k])


def make(name):
    c = workloads.config(name)
    t0 = time.time()
    h1v = [np.diag(h).copy() for h in c["H1"]]   # the perturbations are diagonal
    r = oracle.canonical_response(c["H0"], h1v, None, c["beta"], c["Ne"], c["n"], order=c["order"])
    ii, jj = sample_positions(c["N"])
    out = dict(
        N=c["N"], beta=c["beta"], Ne=c["Ne"], n=c["n"], order=c["order"], dirs=len(h1v),
        i=ii, j=jj, mu0=r["mu0"], mu1=np.array(r["mu1"]), mu2=np.array(r["mu2"]),
        tr_h1p1=np.array(r["tr_h1p1"]), tr_h1p2=np.array(r["tr_h1p2"]),
        P0=r["P0"][ii, jj],
        P1=np.array([p[ii, jj] for p in r["P1"]]),
        P2=np.array([p[ii, jj] for p in r["P2"]]),
        max_P1=np.array([np.abs(p).max() for p in r["P1"]]),
        max_P2=np.array([np.abs(p).max() for p in r["P2"]]),
        seconds=time.time() - t0,
    )
    path = os.path.join(HERE, f"{name}_samples.npz")
    np.savez_compressed(path, **out)
    print(f"{name}: {time.time() - t0:.1f} s -> {path}", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or ["cubic2048", "banded8192"]:
        make(name)
