"""Oracle reference for the plane slab of the Re_tau = 5300 share (8192 x 6144 per plane).

Runs only the oracle (float64, CPU): for two of the 48 planes of the slab, the
seeded spectra of u1, u2, u3, omega1, omega2, omega3 (float32 values, taken
exactly in float64) and their dealiased products H = u x omega on the
12288 x 9216 padded grid.  Stores 4096 seeded (kx, kz) samples of H1, H2, H3
per plane in tests/golden/c3_planes.npz.
Run: python tests/golden/make_c3_golden.py   (about 2 min, ~16 GB RAM)
"""
import os
import sys
import time
import types

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import kmm  # noqa: E402

PLANES = (0, 47)
NS = 4096


def main(out=os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_planes.npz")):
    c = synth.C3_PLANES
    n1, n3 = c["n1"], c["n3"]
    S = types.SimpleNamespace(n1=n1, n3=n3, p1=3 * n1 // 2, p3=3 * n3 // 2)
    g = np.random.default_rng(5300)
    res = {"planes": np.array(PLANES)}
    t0 = time.time()
    for p in PLANES:
        fields = [f.astype(np.complex128)[None] for f in synth.c3_plane_fields(p, n1, n3, c["cfg"])]
        H = kmm.nonlinear(S, fields)
        del fields
        ik, iz = g.integers(0, n1 // 2, NS), g.integers(0, n3, NS)
        iz[iz == n3 // 2] = 0
        res[f"p{p}_ik"], res[f"p{p}_iz"] = ik, iz
        res[f"p{p}_H"] = np.stack([h[0, ik, iz] for h in H])
        res[f"p{p}_Hnorm"] = np.array([np.linalg.norm(h) for h in H])
        del H
        print(f"plane {p} {time.time() - t0:.0f}s", flush=True)
    np.savez_compressed(out, **res)
    print("wrote", out)


if __name__ == "__main__":
    main()
