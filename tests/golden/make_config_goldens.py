#!/usr/bin/env python3
"""Write the oracle goldens of the storage-precision and adjoint configurations.

Calls only the FP64 oracle (``oracle/``) and the seeded input recipes
(``lbm_inputs``); nothing here touches the GPU path.  Run from the repository
root:

    python tests/golden/make_config_goldens.py [decay] [adjoint] [--workers W]

Outputs (JSON text, one file per case):

* ``decay32_d3q27.json``, ``decay32_d3q15.json`` -- the decaying random-phase
  field on a reduced 32^3 periodic lattice: F = 0, rho = 1, solenoidal
  velocity with shells 1..8 and E ~ s^-5/3, per-component rms 0.03 (seed 7),
  1000 steps; D3Q27 at shear rate 1.9, D3Q15 at 1.6, all other rates 1.  The
  mean kinetic energy (1/N) sum |rho u|^2 / (2 rho) of the pre-collision state
  every 10 steps, the FP64 mass at steps 0 and 1000, and the final velocity
  (Eq. velocitycalculation) at 512 seeded nodes.
* ``adjoint32_d3q27.json`` -- the differentiable run on a reduced 32^3
  periodic D3Q27 lattice: Taylor-Green start (k0 = 2 pi / 32, u0 = 0.02),
  force field N(0, (1e-6)^2) per node and component (seed 2024), shear rate
  1.6, others 1, 200 steps; loss = mean kinetic energy of fbar(200) (rho u
  including F/2).  Complex-step derivatives of the loss (the step is rational
  in its inputs, so Im L(p + i h)/h is exact to rounding): along a seeded unit
  direction v of the force field (seed 99), at four seeded single entries of
  the force field, and with respect to the shear rate (omega_4..omega_8
  moved together).

The collision is the plain moment-matrix definition of Sec. 7 and Sec. 8 (with
Appendix G for D3Q15), the streaming Eq. cascadedstreaming1, the initial
state f^eq - S/2 of Sec. 4.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import lbm_inputs as inp  # noqa: E402
from oracle import lbm  # noqa: E402
from oracle.lattice import D3Q15, D3Q27  # noqa: E402
from oracle.pool import Pool  # noqa: E402

H = 1e-30
CMD = "python tests/golden/make_config_goldens.py"


def _rates(q, shear):
    return [shear] * 5 + [1.0] * (q - 9)


def _velocity(lat, f, F):
    _, u = lbm.macroscopic_fields(lat, f, F)
    return u


def decay(pool, lat, shear, n=32, steps=1000, every=10, seed=7, nsample=512):
    q = lat.Q
    u0 = inp.random_spectrum_velocity(n, seed=seed)
    F = np.zeros(3)
    om = _rates(q, shear)
    f = lbm.initial_state(lat, np.ones((n, n, n)), u0, F)
    ke = [float(lbm.kinetic_energy(lat, f, F))]
    mass0 = float(lbm.totals(lat, f, F)[0])
    t0 = time.time()
    for s in range(1, steps + 1):
        f = pool.step(lat, f, F, om)
        if s % every == 0:
            ke.append(float(lbm.kinetic_energy(lat, f, F)))
        if s % 100 == 0:
            print(f"decay D3Q{q}: step {s}, KE {ke[-1]:.6e}, {time.time() - t0:.0f} s", flush=True)
    mass1 = float(lbm.totals(lat, f, F)[0])
    u = _velocity(lat, f, F)
    rng = np.random.default_rng(12345)
    nodes = rng.choice(n**3, size=nsample, replace=False)
    z, rem = np.divmod(nodes, n * n)
    y, x = np.divmod(rem, n)
    return {
        "what": f"D3Q{q} {n}^3 periodic decaying random-phase field, FP64 oracle",
        "recipe": {"n": n, "q": q, "steps": steps, "ke_every": every, "field": "random_spectrum_velocity",
                   "field_seed": seed, "shells": [1, 8], "slope": -5.0 / 3.0, "rms": 0.03, "rho0": 1.0,
                   "force": [0.0, 0.0, 0.0], "rates": om, "shear": shear, "attractor": "literal"},
        "source": "oracle/ (Sec. 7, Sec. 8, Appendix G; streaming Eq. cascadedstreaming1; initial state Sec. 4); "
                  "kinetic energy of the pre-collision state with rho u from Eq. velocitycalculation",
        "command": CMD + " decay",
        "ke": ke,
        "mass": [mass0, mass1],
        "sample_nodes": [[int(a), int(b), int(c)] for a, b, c in zip(z, y, x)],
        "sample_u": [[float(u[k, a, b, c]) for k in range(3)] for a, b, c in zip(z, y, x)],
    }


def _loss(pool, lat, rho0, u0, F, om, steps):
    f = lbm.initial_state(lat, rho0, u0, F)
    f = pool.run(lat, f, F, om, steps)
    return lbm.kinetic_energy(lat, f, F)


def adjoint(pool, n=32, steps=200, shear=1.6):
    lat = D3Q27
    q = 27
    rho0 = np.ones((n, n, n))
    u0 = inp.taylor_green(n, 0.02)
    F = inp.gaussian_force((n, n, n), 1e-6, 2024)
    om = _rates(q, shear)
    v = inp.gaussian_force((n, n, n), 1.0, 99)
    v /= np.sqrt((v * v).sum())
    rng = np.random.default_rng(4242)
    entries = [[int(rng.integers(3)), int(rng.integers(n)), int(rng.integers(n)), int(rng.integers(n))]
               for _ in range(4)]
    t0 = time.time()
    # along v
    Lc = _loss(pool, lat, rho0, u0, F + 1j * H * v, om, steps)
    loss = float(Lc.real)
    d_v = float(Lc.imag / H)
    print(f"adjoint: loss {loss:.12e}, dL/dF.v {d_v:.12e} ({time.time() - t0:.0f} s)", flush=True)
    # shear rate (omega_4..omega_8 together)
    omc = [complex(w) + (1j * H if b < 5 else 0) for b, w in enumerate(om)]
    d_shear = float(_loss(pool, lat, rho0, u0, F.astype(complex), omc, steps).imag / H)
    print(f"adjoint: dL/domega_shear {d_shear:.12e} ({time.time() - t0:.0f} s)", flush=True)
    d_entries = []
    for c, z, y, x in entries:
        Fc = F.astype(complex)
        Fc[c, z, y, x] += 1j * H
        d_entries.append(float(_loss(pool, lat, rho0, u0, Fc, om, steps).imag / H))
        print(f"adjoint: dL/dF[{c},{z},{y},{x}] {d_entries[-1]:.12e} ({time.time() - t0:.0f} s)", flush=True)
    return {
        "what": f"D3Q27 {n}^3 periodic, {steps} steps, loss = mean kinetic energy of fbar({steps}); "
                "FP64 oracle, complex-step derivatives (h = 1e-30)",
        "recipe": {"n": n, "q": q, "steps": steps, "u0": "taylor_green(n, 0.02)", "rho0": 1.0,
                   "force": "gaussian_force((n, n, n), 1e-6, 2024)", "rates": om, "shear": shear,
                   "direction": "gaussian_force((n, n, n), 1.0, 99) normalised to unit L2",
                   "attractor": "literal"},
        "source": "oracle/ (Sec. 7, Sec. 8; streaming Eq. cascadedstreaming1; initial state Sec. 4); "
                  "loss with rho u from Eq. velocitycalculation",
        "command": CMD + " adjoint",
        "loss": loss,
        "dL_dF_dot_v": d_v,
        "dL_domega_shear": d_shear,
        "entries": entries,
        "dL_dF_entries": d_entries,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", nargs="*", default=["decay", "adjoint"])
    ap.add_argument("--workers", type=int, default=None)
    args = ap.parse_args()
    with Pool(args.workers) as pool:
        print(f"{pool.workers} worker processes", flush=True)
        if "decay" in args.what:
            for lat, shear in ((D3Q15, 1.6), (D3Q27, 1.9)):
                rec = decay(pool, lat, shear)
                with open(os.path.join(HERE, f"decay32_d3q{lat.Q}.json"), "w") as fh:
                    json.dump(rec, fh, indent=1)
        if "adjoint" in args.what:
            rec = adjoint(pool)
            with open(os.path.join(HERE, "adjoint32_d3q27.json"), "w") as fh:
                json.dump(rec, fh, indent=1)


if __name__ == "__main__":
    main()
