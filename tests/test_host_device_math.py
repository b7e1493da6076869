"""The library's per-node device math, compiled for the CPU, against the oracle.

tests/host/host_collide.cpp includes the headers the HIP kernels use
(collide_d3q27.hpp, collide_d3q15.hpp) and exports the collision, its
hand-written adjoint and the initial state with C linkage.  Here they are
compared, element by element, with:

* the oracle's plain moment-matrix collision (FP64: 1e-14 relative; FP32:
  the arithmetic's own rounding);
* the oracle's complex-step derivatives for the transposed Jacobians (the
  collision is rational in its inputs, so Im C(x + ih e)/h is exact to
  rounding): populations, force and every relaxation rate;
* the oracle's equilibrium minus half the source for the initial state, and
  its complex-step force derivative.

A sanitizer build (AddressSanitizer + UndefinedBehaviorSanitizer) of the same
code runs pseudo-random nodes of both lattices and must exit clean.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import collision
from oracle.lattice import D3Q15, D3Q27
from paper_1202_6081_amd import build as _b

LATS = {27: D3Q27, 15: D3Q15}
H = 1e-30   # complex step


@pytest.fixture(scope="module")
def lib():
    # (re)build when missing or older than the headers it compiles
    srcs = [_b.HOST_SRC] + [os.path.join(_b.CSRC, n) for n in os.listdir(_b.CSRC) if n.endswith(".hpp")]
    if not os.path.exists(_b.HOST_LIB) or os.path.getmtime(_b.HOST_LIB) < max(map(os.path.getmtime, srcs)):
        _b.build_host_math()
    L = ctypes.CDLL(_b.HOST_LIB)
    dp, fp, i, d = (ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float), ctypes.c_int,
                    ctypes.c_double)
    L.hc_collide_f64.argtypes = [i, dp, dp, dp, i, dp]
    L.hc_collide_f32.argtypes = [i, fp, fp, dp, i, fp]
    L.hc_collide_adj_f64.argtypes = [i, dp, dp, dp, i, dp, dp, dp, dp]
    L.hc_initial_f64.argtypes = [i, d, dp, dp, dp]
    L.hc_initial_adj_force_f64.argtypes = [i, dp, dp, dp]
    for fn in (L.hc_collide_f64, L.hc_collide_f32, L.hc_collide_adj_f64, L.hc_initial_f64,
               L.hc_initial_adj_force_f64):
        fn.restype = None
    return L


def _p(a, ct=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _node(q, rng, umax=0.1, force=1e-3, dev=1e-3):
    lat = LATS[q]
    rho = rng.uniform(0.9, 1.1)
    u = rng.uniform(-umax, umax, 3)
    f = collision.equilibrium(lat, np.array(rho), u) + rng.uniform(-dev, dev, q)
    F = rng.uniform(-force, force, 3)
    om = rng.uniform(0.2, 1.95, q - 4)
    return f, F, om


def _host_collide(lib, q, f, F, om, pm):
    out = np.empty(q)
    lib.hc_collide_f64(q, _p(np.ascontiguousarray(f)), _p(np.ascontiguousarray(F)), _p(om), pm, _p(out))
    return out


@pytest.mark.parametrize("pm", [0, 1])
@pytest.mark.parametrize("q", [27, 15])
def test_collide_f64_matches_oracle(lib, q, pm):
    rng = np.random.default_rng(100 + q + pm)
    for _ in range(25):
        f, F, om = _node(q, rng)
        ref = collision.collide(LATS[q], f, F, list(om), per_mass=bool(pm))
        got = _host_collide(lib, q, f, F, om, pm)
        assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("q", [27, 15])
def test_collide_f64_far_from_equilibrium(lib, q):
    # large velocity, force and deviations: every moment of every order is
    # exercised well away from its attractor
    rng = np.random.default_rng(7 + q)
    for pm in (0, 1):
        f, F, om = _node(q, rng, umax=0.3, force=0.05, dev=0.02)
        ref = collision.collide(LATS[q], f, F, list(om), per_mass=bool(pm))
        got = _host_collide(lib, q, f, F, om, pm)
        assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("q", [27, 15])
def test_collide_f32_within_its_rounding(lib, q):
    rng = np.random.default_rng(300 + q)
    for pm in (0, 1):
        for _ in range(10):
            f, F, om = _node(q, rng)
            f32, F32 = f.astype(np.float32), F.astype(np.float32)
            ref = collision.collide(LATS[q], f32.astype(np.float64), F32.astype(np.float64), list(om),
                                    per_mass=bool(pm))
            out = np.empty(q, dtype=np.float32)
            lib.hc_collide_f32(q, _p(f32, ctypes.c_float), _p(F32, ctypes.c_float), _p(om), pm,
                               _p(out, ctypes.c_float))
            # a few hundred operations of relative size 2^-24 on O(1) moments
            assert np.abs(out.astype(np.float64) - ref).max() <= 2e-6


def _complex_step_vjp(q, f, F, om, pm, g):
    """g^T dC/d(f, F, omega) by complex steps of the oracle's collision."""
    lat = LATS[q]
    gf, gF, gw = np.zeros(q), np.zeros(3), np.zeros(q - 4)
    for a in range(q):
        fc = f.astype(complex)
        fc[a] += 1j * H
        gf[a] = g @ (collision.collide(lat, fc, F.astype(complex), list(om.astype(complex)),
                                       per_mass=bool(pm)).imag / H)
    for k in range(3):
        Fc = F.astype(complex)
        Fc[k] += 1j * H
        gF[k] = g @ (collision.collide(lat, f.astype(complex), Fc, list(om.astype(complex)),
                                       per_mass=bool(pm)).imag / H)
    for b in range(q - 4):
        oc = om.astype(complex)
        oc[b] += 1j * H
        gw[b] = g @ (collision.collide(lat, f.astype(complex), F.astype(complex), list(oc),
                                       per_mass=bool(pm)).imag / H)
    return gf, gF, gw


@pytest.mark.parametrize("pm", [0, 1])
@pytest.mark.parametrize("q", [27, 15])
def test_collide_adjoint_matches_complex_step(lib, q, pm):
    rng = np.random.default_rng(500 + q + pm)
    for _ in range(3):
        f, F, om = _node(q, rng, umax=0.2, force=0.01, dev=0.01)
        g = rng.standard_normal(q)
        ref_f, ref_F, ref_w = _complex_step_vjp(q, f, F, om, pm, g)
        gout, gF, gw = np.empty(q), np.zeros(3), np.zeros(q - 4)
        lib.hc_collide_adj_f64(q, _p(f), _p(F), _p(om), pm, _p(g), _p(gout), _p(gF), _p(gw))
        assert np.abs(gout - ref_f).max() <= 1e-12 * np.abs(ref_f).max()
        assert np.abs(gF - ref_F).max() <= 1e-12 * np.abs(ref_F).max()
        assert np.abs(gw - ref_w).max() <= 1e-12 * max(np.abs(ref_w).max(), 1e-300)


@pytest.mark.parametrize("q", [27, 15])
def test_initial_state_matches_oracle(lib, q):
    rng = np.random.default_rng(900 + q)
    lat = LATS[q]
    for _ in range(20):
        rho = rng.uniform(0.9, 1.1)
        u = rng.uniform(-0.15, 0.15, 3)
        F = rng.uniform(-1e-2, 1e-2, 3)
        ref = collision.equilibrium(lat, np.array(rho), u) - 0.5 * collision.source(lat, F, u)
        out = np.empty(q)
        lib.hc_initial_f64(q, rho, _p(u), _p(F), _p(out))
        assert np.abs(out - ref).max() <= 1e-15 * np.abs(ref).max() * 10


@pytest.mark.parametrize("q", [27, 15])
def test_initial_state_force_adjoint_matches_complex_step(lib, q):
    rng = np.random.default_rng(950 + q)
    lat = LATS[q]
    for _ in range(4):
        u = rng.uniform(-0.15, 0.15, 3)
        F = rng.uniform(-1e-2, 1e-2, 3)
        lam = rng.standard_normal(q)
        ref = np.zeros(3)
        for k in range(3):
            Fc = F.astype(complex)
            Fc[k] += 1j * H
            init = collision.equilibrium(lat, np.array(1.0 + 0j), u.astype(complex)) \
                - 0.5 * collision.source(lat, Fc, u.astype(complex))
            ref[k] = lam @ (init.imag / H)
        gF = np.zeros(3)
        lib.hc_initial_adj_force_f64(q, _p(u), _p(lam), _p(gF))
        assert np.abs(gF - ref).max() <= 1e-13 * np.abs(ref).max()


def test_sanitizer_build_runs_clean():
    exe = _b.build_host_sanitized()
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out
    assert "runtime error" not in out and "AddressSanitizer" not in out, out
    assert "0 failures" in res.stdout
