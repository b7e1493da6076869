#!/usr/bin/env python3
"""Throughput of the fused D3Q27 central-moment LBM step on one MI355X.

Workload (one "step" = one pull-stream + collide + force pass over the whole
lattice): D3Q27, 512^3 periodic, FP32 storage and arithmetic, Kolmogorov body
force field F_x = 1e-6 sin(2 pi 4 y / 512) (read as an FP32 field, 12 B/node),
shear rate omega_4..omega_8 = 1.9, all other rates 1, fluid at rest initially.
Synthetic inputs, no dataset.

Prints ONE JSON line: MLUPS (whole job), the HBM roofline of the step kernel
(algorithmic 228 B per node update: 27 FP32 loads + 27 FP32 stores + 3 FP32
force loads), the FP64 CPU oracle timed on a bounded sample, the
adjoint/forward time ratio of a 100-step checkpointed adjoint, and the
per-launch step time of every lattice/storage variant on the same workload,
two-buffer and in-place, of the FP32 adjoint step of both lattices, and
(`walls`) of the step (two-buffer and in place), the adjoint step and the
wall-layout sensitivity of the same workload inside a square duct.

Accuracy, measured in the same run: every variant's state after its timed
steps against the FP64 variant's (velocity relative L2, kinetic energy), the
count of non-finite stored populations of every final state, the FP16
deviations' subnormal fraction, and (`accuracy`) every variant and the
FP64/FP32 adjoint on the CPU-baseline sample against the oracle's own result
of that sample, which the CPU-baseline leg computes beside its timing.
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline, D3Q27 512^3 FP32 step; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
BYTES_PER_NODE = 27 * 4 * 2 + 3 * 4
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_step_d3q27_f32_512_counters.json")
KERNEL_SOURCES = ["paper_1202_6081_amd/csrc/kernels.hip", "paper_1202_6081_amd/csrc/collide_d3q27.hpp",
                  "paper_1202_6081_amd/csrc/lattice.hpp", "paper_1202_6081_amd/csrc/kernels.hpp"]


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


PROBE = os.path.join(ROOT, "paper_1202_6081_amd", "hbm_probe")


def hbm_ceiling(n):
    """The rates this device sustains for the step's memory traffic with no
    arithmetic, and for plain streams (paper_1202_6081_amd/hbm_probe, run in a
    process of its own before this one allocates anything): the ceiling the
    step's roofline fraction is read against.  None where the probe's launch
    shape does not cover n or it is not built."""
    if n % 256 != 0 or n > 1024 or not os.path.exists(PROBE):
        return None
    try:
        res = subprocess.run([PROBE, str(n)], capture_output=True, text=True, timeout=300)
        if res.returncode == 0:
            return json.loads(res.stdout.strip().splitlines()[-1])
        print("hbm_probe failed (no ceiling reported): " + res.stderr[-500:], file=sys.stderr)
    except (OSError, ValueError, IndexError, subprocess.TimeoutExpired) as e:
        print(f"hbm_probe failed (no ceiling reported): {e}", file=sys.stderr)
    return None


def measured_traffic(n_nodes):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    try:
        with open(COUNTERS_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash() or rec.get("nodes") != n_nodes:
        return None
    return rec.get("hbm_bytes_per_dispatch")


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(seconds_target=12.0, n=48, max_steps=48, adjoint_steps=8):
    """The FP64 oracle on the host's cores, on a bounded sample of the same
    workload: an n^3 D3Q27 periodic box from rest with the benchmark's rates
    and Kolmogorov force F_x = 1e-6 sin(2 pi 4 y / n), stepped until about
    `seconds_target` seconds have passed.  The oracle code is unchanged; its
    per-node collisions are spread over a process pool (oracle/pool.py), one
    worker per host CPU up to 16.

    Also returns, untimed, the oracle references of the accuracy checks on the
    same sample: the final D3Q27 state, the same number of D3Q15 steps, and the
    complex-step derivative of the mean kinetic energy after `adjoint_steps`
    steps along the unit direction of the force field itself."""
    import numpy as np
    from oracle import lbm
    from oracle.lattice import D3Q15, D3Q27
    from oracle.pool import Pool
    import lbm_inputs as inp
    F = inp.kolmogorov_force(n, waves=4)
    om27 = [1.9] * 5 + [1.0] * 18
    om15 = [1.9] * 5 + [1.0] * 6
    rho0, u0 = np.ones((n, n, n)), np.zeros((3, n, n, n))
    with Pool() as pool:
        f = lbm.initial_state(D3Q27, rho0, u0, F)
        f = pool.step(D3Q27, f, F, om27)             # starts the workers (untimed)
        t0 = time.perf_counter()
        steps = 0
        while True:
            f = pool.step(D3Q27, f, F, om27)
            steps += 1
            el = time.perf_counter() - t0
            if el > seconds_target or steps >= max_steps:
                break
        total = steps + 1
        record = {"value": n**3 * steps / el / 1e6, "unit": "MLUPS", "cores": pool.workers, "kind": "oracle",
                  "host_cpus": os.cpu_count(), "cpu_model": _cpu_model(),
                  "sample": f"{steps} timed step(s) of a {n}^3 D3Q27 periodic box from rest, FP64 NumPy oracle, "
                            f"collisions over {pool.workers} worker processes, Kolmogorov force, shear rate 1.9 "
                            f"({el:.1f} s)"}
        g = lbm.initial_state(D3Q15, rho0, u0, F)
        g = pool.run(D3Q15, g, F, om15, total)
        v = F / np.sqrt((F * F).sum())             # along the force itself: d L / d (force amplitude)
        h = 1e-30
        Fc = F + 1j * h * v
        fc = pool.run(D3Q27, lbm.initial_state(D3Q27, rho0, u0, Fc), Fc, om27, adjoint_steps)
        loss = lbm.kinetic_energy(D3Q27, fc, Fc)
    ref = {"n": n, "steps": total, "F": F, "f27": f, "f15": g,
           "u27": lbm.macroscopic_fields(D3Q27, f, F)[1], "u15": lbm.macroscopic_fields(D3Q15, g, F)[1],
           "adjoint_steps": adjoint_steps, "direction": v, "loss": float(loss.real),
           "dL_dF_dot_v": float(loss.imag / h)}
    return record, ref


def _rel_l2(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def accuracy_vs_oracle(ref):
    """Every lattice/storage variant on the cpu_baseline sample against the
    oracle's result of the same steps (velocity relative L2, largest population
    error), and the FP64 and FP32 adjoint gradients along the sample's direction
    against the oracle's complex step."""
    import numpy as np
    import torch
    from paper_1202_6081_amd import autograd as ag
    from paper_1202_6081_amd import cmlbm
    n, steps, dev = ref["n"], ref["steps"], torch.device("cuda", 0)
    out = {"sample": f"{n}^3 D3Q27/D3Q15 periodic box, the benchmark's recipe, {steps} steps from rest; "
                     f"adjoint: {ref['adjoint_steps']} steps, loss = mean kinetic energy, derivative along the "
                     "force field's own direction; FP32 gradient field also against the FP64 one (relative L2)",
           "variants": []}
    for q in (27, 15):
        fo, uo = ref[f"f{q}"], ref[f"u{q}"]
        for prec in (cmlbm.F64, cmlbm.F32, cmlbm.F32_F16DEV, cmlbm.F32_BF16DEV):
            sim = cmlbm.Sim(q, n, n, n, prec)
            sim.set_rates([1.9] * 5 + [1.0] * (q - 9))
            sim.set_force(torch.from_numpy(ref["F"]).to(dev, sim.real))
            a, _ = sim.init_equilibrium(torch.ones((n, n, n), device=dev, dtype=sim.real),
                                        torch.zeros((3, n, n, n), device=dev, dtype=sim.real))
            last = sim.run(a, sim.populations(), steps)
            fg = sim.gather(last).double().cpu().numpy()
            ug = sim.macroscopic(last)[1].double().cpu().numpy()
            out["variants"].append({"lattice": f"D3Q{q}", "storage": cmlbm.PRECISION_NAMES[prec],
                                    "u_rel_l2": _rel_l2(ug, uo),
                                    "f_max_abs_err": float(np.abs(fg - fo).max())})
            del sim, a, last
    v = ref["direction"]
    adj = {"oracle_dL_dF_dot_v": ref["dL_dF_dot_v"]}
    grads = {}
    for prec in (cmlbm.F64, cmlbm.F32):
        sim = cmlbm.Sim(27, n, n, n, prec)
        F = torch.from_numpy(ref["F"]).to(dev, sim.real).requires_grad_(True)
        omega = torch.tensor([1.9] * 5 + [1.0] * 18, dtype=torch.float64, requires_grad=True)
        rho0 = torch.ones((n, n, n), device=dev, dtype=sim.real)
        u0 = torch.zeros((3, n, n, n), device=dev, dtype=sim.real)
        pre = ag.run(sim, rho0, u0, F, omega, ref["adjoint_steps"], every=ref["adjoint_steps"])
        ag.kinetic_energy(sim, pre, F).backward()
        # F.grad: the run's adjoint plus the loss's own dependence on F (rho u includes F/2)
        grads[prec] = F.grad.double().cpu().numpy()
        d = float((grads[prec] * v).sum())
        adj[f"{cmlbm.PRECISION_NAMES[prec]}_rel_err"] = abs(d / ref["dL_dF_dot_v"] - 1)
        del sim, F, pre
    adj["f32_grad_rel_l2_vs_f64"] = _rel_l2(grads[cmlbm.F32], grads[cmlbm.F64])
    out["adjoint"] = adj
    torch.cuda.empty_cache()
    return out


def _velocity_and_ke(sim, f_post):
    """Velocity (FP64, on the device) and mean kinetic energy of the state
    pulled from f_post, from the library's own read-out."""
    rho, u = sim.macroscopic(f_post)
    u = u.double()
    ke = float((0.5 * rho.double() * (u * u).sum(dim=0)).mean())
    del rho
    return u, ke


def _f16_exposure(buf):
    """Fractions of the stored FP16 deviations that are subnormal (nonzero,
    below 2^-14 = 6.1e-5 in magnitude) and that are zero."""
    import torch
    bits = buf.view(torch.int16).reshape(-1)
    expo = (bits >> 10) & 0x1F
    mant = bits & 0x3FF
    sub = int(((expo == 0) & (mant != 0)).sum())
    zero = int(((expo == 0) & (mant == 0)).sum())
    return sub / bits.numel(), zero / bits.numel()


def variant_sweep(n, steps=30, warmup=3):
    """Per-launch step time of every lattice and storage variant on the same
    512^3 workload (events around each launch on its stream), for the
    two-buffer step and for the in-place step (mean of its two phases).  Each
    variant's state after its warmup + timed two-buffer steps is compared with
    the FP64 variant's state after the same steps (velocity relative L2, mean
    kinetic energy), its non-finite stored populations are counted, and for
    FP16 deviation storage the stored values' subnormal and zero fractions."""
    import torch
    import lbm_inputs as inp
    from paper_1202_6081_amd import cmlbm
    dev = torch.device("cuda", 0)
    out = []
    for q in (27, 15):
        u64 = ke64 = None
        for prec, name, tb in ((cmlbm.F64, "f64", 8), (cmlbm.F32, "f32", 4), (cmlbm.F32_F16DEV, "f16dev", 2),
                               (cmlbm.F32_BF16DEV, "bf16dev", 2)):
            sim = cmlbm.Sim(q, n, n, n, prec)
            sim.set_rates([1.9] * 5 + [1.0] * (q - 9))
            sim.set_force(torch.from_numpy(inp.kolmogorov_force(n, amplitude=1e-6, waves=4)).to(dev, sim.real))
            a, b = sim.populations(), sim.populations()
            pre = sim.real_populations()
            sim.init_equilibrium(torch.ones((n, n, n), device=dev, dtype=sim.real),
                                 torch.zeros((3, n, n, n), device=dev, dtype=sim.real), f_post=a, f_pre=pre)
            bufs = [a, b]
            for i in range(warmup):
                sim.step(bufs[i & 1], bufs[(i + 1) & 1])
            ms = _launch_ms(lambda i: sim.step(bufs[(warmup + i) & 1], bufs[(warmup + i + 1) & 1]), steps)
            last = bufs[(warmup + steps) & 1]
            u, ke = _velocity_and_ke(sim, last)
            acc = {"steps": warmup + steps, "ke": ke, "nonfinite_populations": sim.check_finite(last)}
            if prec == cmlbm.F64:
                u64, ke64 = u, ke
            else:
                acc["u_rel_l2_vs_f64"] = float(torch.linalg.vector_norm(u - u64) / torch.linalg.vector_norm(u64))
                acc["ke_rel_err_vs_f64"] = abs(ke / ke64 - 1)
                del u
            if prec == cmlbm.F32_F16DEV:
                acc["f16_subnormal_frac"], acc["f16_zero_frac"] = _f16_exposure(last)
            del last
            # the in-place (one-buffer) step from the same initial state
            sim.import_populations(pre, b)
            del pre
            for i in range(warmup + (warmup & 1)):
                sim.step_inplace(b, i & 1)
            t_in = _launch_ms(lambda i: sim.step_inplace(b, i & 1), 2 * (steps // 2), per_launch=True)
            ms_even, ms_odd = sum(t_in[0::2]) / len(t_in[0::2]), sum(t_in[1::2]) / len(t_in[1::2])
            ms_in = (ms_even + ms_odd) / 2
            bpn = q * tb * 2 + 3 * (8 if prec == cmlbm.F64 else 4)
            gbs = bpn * n**3 / (ms * 1e-3) / 1e9
            gbs_in = bpn * n**3 / (ms_in * 1e-3) / 1e9
            out.append({"lattice": f"D3Q{q}", "storage": name, "ms": round(ms, 4),
                        "MLUPS": round(n**3 / (ms * 1e-3) / 1e6, 1), "bytes_per_node": bpn,
                        "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4), "accuracy": acc,
                        "inplace": {"ms": round(ms_in, 4), "ms_collide_phase": round(ms_even, 4),
                                    "ms_scatter_phase": round(ms_odd, 4),
                                    "MLUPS": round(n**3 / (ms_in * 1e-3) / 1e6, 1),
                                    "frac": round(gbs_in / HBM_PEAK_GBS, 4),
                                    "state_GiB": round(q * tb * n**3 / 2**30, 2)}})
            del a, b, bufs, sim
            torch.cuda.empty_cache()
        del u64
    return out


def adjoint_sweep(n, launches=6):
    """Per-call time of one FP32 adjoint step (the adjoint kernel and its two
    small reductions) for both lattices on the 512^3 workload: algorithmic
    bytes per node 3 Q 4 (pull of the forward state, reverse gather of lambda,
    store of lambda) + 12 (force field) + 48 (FP64 dL/dF read-modify-write)."""
    import torch
    import lbm_inputs as inp
    from paper_1202_6081_amd import cmlbm
    dev = torch.device("cuda", 0)
    out = []
    for q in (27, 15):
        sim = cmlbm.Sim(q, n, n, n, cmlbm.F32)
        sim.set_rates([1.9] * 5 + [1.0] * (q - 9))
        sim.set_force(torch.from_numpy(inp.kolmogorov_force(n, amplitude=1e-6, waves=4)).to(dev, torch.float32))
        x = sim.populations()
        lam_a, lam_b = sim.real_populations(), sim.real_populations()
        sim.init_equilibrium(torch.ones((n, n, n), device=dev), torch.zeros((3, n, n, n), device=dev),
                             f_post=x, f_pre=lam_a)
        dLdF = torch.zeros((3, n, n, n), dtype=torch.float64, device=dev)
        dLdw = torch.zeros(q - 4, dtype=torch.float64, device=dev)
        bufs = [lam_a, lam_b]
        sim.adjoint_step(x, lam_a, lam_b, dLdF, dLdw)
        ms = _launch_ms(lambda i: sim.adjoint_step(x, bufs[i & 1], bufs[(i + 1) & 1], dLdF, dLdw), launches)
        bpn = 3 * q * 4 + 12 + 48
        gbs = bpn * n**3 / (ms * 1e-3) / 1e9
        out.append({"lattice": f"D3Q{q}", "storage": "f32", "ms": round(ms, 4), "bytes_per_node": bpn,
                    "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)})
        del sim, x, lam_a, lam_b, bufs, dLdF
        torch.cuda.empty_cache()
    return out


def wall_sweep(n, launches=6):
    """Per-call time of the masked FP32 D3Q27 step, adjoint step and wall-layout
    sensitivity (gather form) on the 512^3 workload inside a square duct
    (solid planes y, z in {0, n-1}, as in Sec. 9), with algorithmic bytes per
    node over all n^3 nodes: step 228 and adjoint 384 as without walls; the
    wall term 26 x 4 (collided state) + 26 x 4 (lambda) + 16 (FP64 dL/dphi
    read-modify-write) = 224: each lambda value enters twice, as lambda_a of
    its own node and as lambda_abar of the neighbour it feeds, and counts once."""
    import torch
    import lbm_inputs as inp
    from paper_1202_6081_amd import cmlbm
    dev = torch.device("cuda", 0)
    q = 27
    sim = cmlbm.Sim(q, n, n, n, cmlbm.F32)
    sim.set_rates([1.9] * 5 + [1.0] * (q - 9))
    sim.set_force(torch.from_numpy(inp.kolmogorov_force(n, amplitude=1e-6, waves=4)).to(dev, torch.float32))
    sim.set_mask(torch.from_numpy(inp.duct_mask(n, n, n)))
    x, x1 = sim.populations(), sim.populations()
    lam_a, lam_b = sim.real_populations(), sim.real_populations()
    sim.init_equilibrium(torch.ones((n, n, n), device=dev), torch.zeros((3, n, n, n), device=dev),
                         f_post=x, f_pre=lam_a)
    sim.step(x, x1)
    dLdF = torch.zeros((3, n, n, n), dtype=torch.float64, device=dev)
    dLdw = torch.zeros(q - 4, dtype=torch.float64, device=dev)
    dphi = torch.zeros((n, n, n), dtype=torch.float64, device=dev)
    bufs, xs = [lam_a, lam_b], [x, x1]
    out = {"workload": f"D3Q27 {n}^3 FP32, square duct along x (solid planes y, z in {{0, {n - 1}}}), "
                       "Kolmogorov force field, shear rate 1.9"}
    for name, bpn, launch in (
            ("step", 228, lambda i: sim.step(xs[i & 1], xs[(i + 1) & 1])),
            ("adjoint_step", 384, lambda i: sim.adjoint_step(x, bufs[i & 1], bufs[(i + 1) & 1], dLdF, dLdw)),
            ("wall_sensitivity", 224, lambda i: sim.wall_sensitivity_post(x1, lam_a, dphi))):
        launch(0)
        ms = _launch_ms(launch, launches)
        gbs = bpn * n**3 / (ms * 1e-3) / 1e9
        out[name] = {"ms": round(ms, 4), "bytes_per_node": bpn, "GBs": round(gbs, 1),
                     "frac": round(gbs / HBM_PEAK_GBS, 4)}
    del x, x1, lam_a, lam_b, bufs, xs, dLdF, dphi
    torch.cuda.empty_cache()
    # the same duct stepped in place (one buffer: collide phase, scatter phase)
    b = sim.init_equilibrium_inplace(torch.ones((n, n, n), device=dev), torch.zeros((3, n, n, n), device=dev))
    for i in range(2):
        sim.step_inplace(b, i & 1)
    t_in = _launch_ms(lambda i: sim.step_inplace(b, i & 1), 2 * (launches // 2), per_launch=True)
    ms_even, ms_odd = sum(t_in[0::2]) / len(t_in[0::2]), sum(t_in[1::2]) / len(t_in[1::2])
    gbs = 228 * n**3 / ((ms_even + ms_odd) / 2 * 1e-3) / 1e9
    out["inplace"] = {"ms_collide_phase": round(ms_even, 4), "ms_scatter_phase": round(ms_odd, 4),
                      "bytes_per_node": 228, "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    del sim, b
    torch.cuda.empty_cache()
    return out


def _launch_ms(launch, count, per_launch=False):
    """Duration of each of `count` launches (event pair around each on the
    launch stream); their mean, or the list with per_launch."""
    import torch
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(count)]
    torch.cuda.synchronize()
    for i in range(count):
        ev[i][0].record(stream)
        launch(i)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    t = [e0.elapsed_time(e1) for e0, e1 in ev]
    return t if per_launch else sum(t) / count


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed steps first (about 1 s at 512^3: the clocks settle within that)")
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--adjoint-steps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-ceiling", action="store_true", help="skip the HBM rate probe")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the per-variant step timings (both lattices, four storage types)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 4 GiB device buffer 8 times (known bytes, for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the build targets single-GPU runs only "
              "(multi-GPU z-slab decomposition is a design note, not built).", file=sys.stderr)
        sys.exit(2)

    ceiling = None if (args.no_ceiling or args.copy_calibration) else hbm_ceiling(args.n)
    # the oracle's timing and references first, in worker processes of its own,
    # before this process touches the device
    cpu, ref = (None, None) if (args.no_cpu_baseline or args.copy_calibration) else cpu_baseline()

    import torch
    import lbm_inputs as inp
    from paper_1202_6081_amd import cmlbm

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        src = torch.ones(1 << 30, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(8):
            dst.copy_(src)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 8
        print(json.dumps({"copy_bytes_read": 4 << 30, "copy_bytes_written": 4 << 30,
                          "copy_GBs": round(2 * (4 << 30) / dt / 1e9, 1)}), flush=True)
        return
    n = args.n
    N = n**3
    sim = cmlbm.Sim(27, n, n, n, cmlbm.F32)
    sim.set_rates([1.9] * 5 + [1.0] * 18)
    F = torch.from_numpy(inp.kolmogorov_force(n, amplitude=1e-6, waves=4)).to(dev, torch.float32)
    sim.set_force(F)
    del F
    a = sim.populations()
    b = sim.populations()
    rho0 = torch.ones((n, n, n), device=dev, dtype=torch.float32)
    u0 = torch.zeros((3, n, n, n), device=dev, dtype=torch.float32)
    sim.init_equilibrium(rho0, u0, f_post=a, f_pre=b)
    del rho0, u0
    stream = torch.cuda.current_stream()
    bufs = [a, b]
    for i in range(args.warmup):
        sim.step(bufs[i & 1], bufs[(i + 1) & 1])
    k0 = args.warmup
    torch.cuda.synchronize()
    # whole-job time of K steps, and each launch's own duration (event pair on
    # the launch stream around every step) for the kernel roofline
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    start.record(stream)
    for i in range(args.steps):
        j = k0 + i
        ev[i][0].record(stream)
        sim.step(bufs[j & 1], bufs[(j + 1) & 1])
        ev[i][1].record(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    kernel_ms = sum(e0.elapsed_time(e1) for e0, e1 in ev) / args.steps
    last = bufs[(k0 + args.steps) & 1]
    ms_per_step = ms / args.steps
    mlups = N / (ms_per_step * 1e-3) / 1e6
    achieved = BYTES_PER_NODE * N / (kernel_ms * 1e-3) / 1e9
    traffic = measured_traffic(N)
    tot = sim.totals(last)
    torch.cuda.synchronize()
    t_chk = time.perf_counter()
    nonfinite = sim.check_finite(last)      # synchronizes
    check_ms = (time.perf_counter() - t_chk) * 1e3

    result = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"D3Q27 central-moment LBM {n}^3 periodic, FP32, Kolmogorov force field "
                               f"F_x=1e-6 sin(2 pi 4 y/{n}), shear rate 1.9, others 1.0, from rest",
                   "lattice": "D3Q27", "nodes": N, "storage": "f32", "force": "field"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / (kernel_ms * 1e-3) / 1e9, 1),
                     "algorithmic_bytes_per_node": BYTES_PER_NODE, "kernel": "k_step<27,StF32,false>",
                     "kernel_ms_avg": round(kernel_ms, 4)},
        "mass_total_fp64": tot[0],
        "nonfinite_populations": nonfinite,
        "check_finite_ms": round(check_ms, 3),
        "hbm_ceiling": None if ceiling is None else {
            "step_traffic_GBs": ceiling["step_traffic_pull_GBs"],
            "step_traffic_own_node_GBs": ceiling["step_traffic_own_node_GBs"],
            "read_GBs": ceiling["read_GBs"], "write_GBs": ceiling["write_GBs"], "copy_GBs": ceiling["copy_GBs"],
            "kernel_over_ceiling": round(achieved / ceiling["step_traffic_pull_GBs"], 4),
            "adjoint_traffic_GBs": ceiling.get("adjoint_traffic_GBs"),
            "stream_flavours_GBs": ceiling.get("stream_flavours_GBs"),
            "probe": "paper_1202_6081_amd/hbm_probe: plain read/write/copy streams over 4 GiB (best of 4/8/16 B "
                     "per lane, plain/nontemporal/sc1 policies, one-pass or grid-stride), the step's loads and "
                     "stores (27 pull loads, 3 force loads, 27 stores per node) and the adjoint's (384 B per "
                     "node), no arithmetic, same layouts, one node per thread"},
    }
    del a, b, bufs, last
    torch.cuda.empty_cache()
    if not args.no_adjoint:
        from paper_1202_6081_amd import autograd as ag
        result["adjoint"] = ag.benchmark_adjoint_ratio(sim, args.adjoint_steps, forward_ms_per_step=ms_per_step)
        result["adjoint_forward_ratio"] = result["adjoint"]["ratio_backward_over_forward_steps"]
    else:
        result["adjoint"] = None
        result["adjoint_forward_ratio"] = None
    torch.cuda.empty_cache()
    result["variants"] = None if args.no_variants else variant_sweep(n)
    result["adjoint_variants"] = None if args.no_variants else adjoint_sweep(n)
    result["walls"] = None if args.no_variants else wall_sweep(n)
    hc = result["hbm_ceiling"]
    if hc is not None and hc["adjoint_traffic_GBs"] and result["adjoint_variants"]:
        adj27 = next(v for v in result["adjoint_variants"] if v["lattice"] == "D3Q27")
        hc["adjoint_over_ceiling"] = round(adj27["GBs"] / hc["adjoint_traffic_GBs"], 4)
    # the same workload stepped in place (one population buffer)
    result["inplace"] = None if args.no_variants else next(
        v["inplace"] for v in result["variants"] if v["lattice"] == "D3Q27" and v["storage"] == "f32")
    if cpu is not None:
        result["cpu_baseline"] = cpu
        result["accuracy"] = accuracy_vs_oracle(ref)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
