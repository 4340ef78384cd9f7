"""Writes tests/golden/mwa256x768_3d.json: FP64 oracle results of the 3D bispectrum on the
MWA-shaped cube, for the full-size GPU parity test.

    python tests/golden/make_mwa_golden.py [--workers 8]

Inputs (seeded, paper_2506_10526_amd.synth): the 256 x 256 uv x 768 channel cube of 40 kHz
channels at the set-up of Sec. 4 (quadratic field, P ~ k^-2, sigma 0.5, f 0.5), 20 log |k|
shells over 0.003-1.258 Mpc^-1 (Sec. 5), every support cell sampled once; once without flags
and once with channels {0, 16, 31} of every 32-channel block flagged.
Outputs, from the oracle only:
  * T3D: exact integer counts of every candidate triangle (oracle.counts.exact_counts: pair
    convolutions rounded per cell, summed in int64) -- geometry only, the same for both cubes;
  * per cube: B (oracle.estimator.estimate_3d in float64 with those counts), N_eff, and the
    scale norm N_vox sum|F1 F2 F3| / N_eff that the parity test uses for the conditioning of
    each entry (cond = scale / |B|);
  * a checksum of each cube so that the test can tell that it regenerated the same input.
Takes about 20 minutes and 20 GB of memory on 8 cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import bins as ob  # noqa: E402
from oracle import counts as oc  # noqa: E402
from oracle import estimator as oe  # noqa: E402
from paper_2506_10526_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mwa256x768_3d.json")
SEED = 2506


def cube_checksum(V: np.ndarray) -> dict:
    return {"sum_re": float(np.sum(V.real)), "sum_im": float(np.sum(V.imag)), "sum_abs2": float(np.sum(np.abs(V) ** 2))}


def shell_bins(w):
    return ob.make_bins(ob.SHELL_K, w.n, w.nc, w.shell_edges(20), du=w.du, r_mpc=w.r_mpc, rprime=w.rprime, dnu=w.dnu)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    t0 = time.time()
    w2 = synth.config2()
    b = shell_bins(w2)
    T, dev = oc.exact_counts(b, None, workers=args.workers)
    print(f"exact counts: {time.time() - t0:.0f} s, pair-count rounding deviation {dev:.3g}", flush=True)
    out = {
        "recipe": "synth.config2() / synth.config3() cubes, synth.make_cube(seed), 20 log shells "
                  "geomspace(0.003, 1.258, 21) Mpc^-1, no uv mask (every support cell sampled once)",
        "seed": SEED, "n": w2.n, "nc": w2.nc, "edges": [float(x) for x in w2.shell_edges(20)],
        "triangles": b.triangles.tolist(), "T3D": [int(x) for x in T], "pair_count_rounding_dev": dev,
        "cubes": {},
    }
    nvox = w2.nc * w2.n * w2.n
    for name, w in (("unflagged", synth.config2()), ("flagged", synth.config3())):
        t1 = time.time()
        V = synth.make_cube(w, seed=SEED)
        wt = oe.Weights(chan_w=w.chan_w() if w.flags_mod32 else None)
        f = oe.ShellFields(b, V, wt)
        B, T3, neff, S, _ = oe.estimate_3d(b, V, wt, fields=f, counts=T)
        # sum |F1 F2 F3| per triangle (conditioning scale), by pair products
        absf = {}
        A = np.zeros(len(b.triangles))
        for t, (i, j, k) in enumerate(b.triangles):
            for x in (i, j, k):
                if x not in absf:
                    absf[x] = np.abs(f.data(x)).ravel()
            A[t] = float(np.dot(absf[i] * absf[j], absf[k]))
        with np.errstate(divide="ignore", invalid="ignore"):
            scale = np.where(T > 0, nvox * A / np.maximum(neff, 1e-300), 0.0)
        out["cubes"][name] = {
            "flags_mod32": list(w.flags_mod32), "rho3": oe.rho3(wt, w.nc), "checksum": cube_checksum(V),
            "B": [float(x) for x in B], "N_eff": [float(x) for x in neff], "abs_scale": [float(x) for x in scale],
        }
        print(f"{name}: {time.time() - t1:.0f} s", flush=True)
        del f, absf
    with open(OUT, "w") as fh:
        json.dump(out, fh)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
