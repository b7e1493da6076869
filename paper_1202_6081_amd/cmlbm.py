"""ctypes binding of libcmlbm.so (include/cmlbm.h): argument marshalling only.

Each ``cmlbm_*`` function mirrors the C function of the same name; device
buffers are torch tensors on the current HIP device (their ``data_ptr()`` is
passed), streams default to torch's current stream.  Every numerical step runs
in the library's HIP kernels; there is no fallback: importing this module on a
machine without the built library raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcmlbm.so")

D3Q15, D3Q27 = 15, 27
F64, F32, F32_F16DEV, F32_BF16DEV = 0, 1, 2, 3
PRECISION_NAMES = {F64: "f64", F32: "f32", F32_F16DEV: "f16dev", F32_BF16DEV: "bf16dev"}

_lib = None


class CmlbmError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"cmlbm error {code}: {message}")
        self.code = code


def load_library():
    """Load libcmlbm.so (built in-tree by paper_1202_6081_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise CmlbmError(-2, f"{LIB_PATH} is missing: run `python -m paper_1202_6081_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "cmlbm_create": (i, [i, i, i, i, i, ctypes.POINTER(vp)]),
        "cmlbm_destroy": (None, [vp]),
        "cmlbm_set_rates": (i, [vp, ctypes.POINTER(d), i]),
        "cmlbm_set_force_uniform": (i, [vp, d, d, d]),
        "cmlbm_set_force_field": (i, [vp, vp]),
        "cmlbm_set_force_scale": (i, [vp, d]),
        "cmlbm_set_attractor_per_mass": (i, [vp, i]),
        "cmlbm_set_mask": (i, [vp, vp]),
        "cmlbm_init_equilibrium": (i, [vp, vp, vp, vp, vp, vp]),
        "cmlbm_step": (i, [vp, vp, vp, vp]),
        "cmlbm_step_totals": (i, [vp, vp, vp, vp, vp]),
        "cmlbm_step_totals_noalloc": (i, [vp, vp, vp, vp, vp]),
        "cmlbm_run": (i, [vp, vp, vp, i, vp, ctypes.POINTER(i)]),
        "cmlbm_gather_precollision": (i, [vp, vp, vp, vp]),
        "cmlbm_export_populations": (i, [vp, vp, vp, vp]),
        "cmlbm_import_populations": (i, [vp, vp, vp, vp]),
        "cmlbm_macroscopic": (i, [vp, vp, vp, vp, vp]),
        "cmlbm_totals": (i, [vp, vp, ctypes.POINTER(d), vp]),
        "cmlbm_init_equilibrium_inplace": (i, [vp, vp, vp, vp, vp]),
        "cmlbm_step_inplace": (i, [vp, vp, i, vp]),
        "cmlbm_step_inplace_totals": (i, [vp, vp, i, vp, vp]),
        "cmlbm_run_inplace": (i, [vp, vp, i, vp]),
        "cmlbm_macroscopic_pre": (i, [vp, vp, vp, vp, vp]),
        "cmlbm_totals_pre": (i, [vp, vp, ctypes.POINTER(d), vp]),
        "cmlbm_adjoint_step": (i, [vp, vp, vp, vp, vp, vp, vp]),
        "cmlbm_wall_sensitivity": (i, [vp, vp, vp, vp, vp]),
        "cmlbm_wall_sensitivity_post": (i, [vp, vp, vp, vp, vp]),
        "cmlbm_check_finite": (i, [vp, vp, ctypes.POINTER(ctypes.c_int64), vp]),
        "cmlbm_kinetic_energy_sum": (i, [vp, vp, ctypes.POINTER(d), vp]),
        "cmlbm_kinetic_energy_seed": (i, [vp, vp, d, vp, vp, vp]),
        "cmlbm_init_adjoint": (i, [vp, vp, vp, vp, vp]),
        "cmlbm_status_string": (ctypes.c_char_p, [i]),
        "cmlbm_last_error": (ctypes.c_char_p, [vp]),
        "cmlbm_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return ["cmlbm_create", "cmlbm_destroy", "cmlbm_set_rates", "cmlbm_set_force_uniform",
            "cmlbm_set_force_field", "cmlbm_set_force_scale", "cmlbm_set_attractor_per_mass", "cmlbm_set_mask",
            "cmlbm_init_equilibrium", "cmlbm_step", "cmlbm_step_totals", "cmlbm_step_totals_noalloc", "cmlbm_run",
            "cmlbm_gather_precollision",
            "cmlbm_export_populations", "cmlbm_import_populations", "cmlbm_macroscopic", "cmlbm_totals",
            "cmlbm_init_equilibrium_inplace", "cmlbm_step_inplace", "cmlbm_step_inplace_totals",
            "cmlbm_run_inplace", "cmlbm_macroscopic_pre", "cmlbm_totals_pre",
            "cmlbm_adjoint_step", "cmlbm_wall_sensitivity", "cmlbm_wall_sensitivity_post",
            "cmlbm_check_finite", "cmlbm_kinetic_energy_sum", "cmlbm_kinetic_energy_seed",
            "cmlbm_init_adjoint",
            "cmlbm_status_string", "cmlbm_last_error", "cmlbm_version"]


# ----------------------------------------------------------------------------
# marshalling helpers
# ----------------------------------------------------------------------------
def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise CmlbmError(-1, "device buffers must be torch tensors on the GPU")
    if not t.is_contiguous():
        raise CmlbmError(-1, "device buffers must be contiguous")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(code, handle=None):
    if code != 0:
        lib = load_library()
        msg = lib.cmlbm_last_error(handle).decode() if handle is not None else ""
        if not msg:
            msg = lib.cmlbm_status_string(code).decode()
        raise CmlbmError(code, msg)


def real_dtype(precision):
    return torch.float64 if precision == F64 else torch.float32


def storage_dtype(precision):
    return {F64: torch.float64, F32: torch.float32, F32_F16DEV: torch.float16,
            F32_BF16DEV: torch.bfloat16}[precision]


# ----------------------------------------------------------------------------
# one Python function per C entry point
# ----------------------------------------------------------------------------
def cmlbm_create(q, nx, ny, nz, precision):
    lib = load_library()
    h = ctypes.c_void_p()
    code = lib.cmlbm_create(q, nx, ny, nz, precision, ctypes.byref(h))
    if code != 0:
        raise CmlbmError(code, lib.cmlbm_last_error(None).decode())
    return h


def cmlbm_destroy(h):
    load_library().cmlbm_destroy(h)


def cmlbm_set_rates(h, omega):
    arr = (ctypes.c_double * len(omega))(*[float(w) for w in omega])
    _check(load_library().cmlbm_set_rates(h, arr, len(omega)), h)


def cmlbm_set_force_uniform(h, fx, fy, fz):
    _check(load_library().cmlbm_set_force_uniform(h, float(fx), float(fy), float(fz)), h)


def cmlbm_set_force_field(h, F):
    _check(load_library().cmlbm_set_force_field(h, _ptr(F)), h)


def cmlbm_set_force_scale(h, scale):
    _check(load_library().cmlbm_set_force_scale(h, float(scale)), h)


def cmlbm_set_attractor_per_mass(h, per_mass):
    _check(load_library().cmlbm_set_attractor_per_mass(h, int(bool(per_mass))), h)


def cmlbm_set_mask(h, mask):
    _check(load_library().cmlbm_set_mask(h, _ptr(mask)), h)


def cmlbm_init_equilibrium(h, rho, u, f_pre, f_post, stream=None):
    _check(load_library().cmlbm_init_equilibrium(h, _ptr(rho), _ptr(u), _ptr(f_pre), _ptr(f_post),
                                                  _stream(stream)), h)


def cmlbm_step(h, f_in, f_out, stream=None):
    _check(load_library().cmlbm_step(h, _ptr(f_in), _ptr(f_out), _stream(stream)), h)


def cmlbm_step_totals(h, f_in, f_out, totals, stream=None):
    if totals.dtype != torch.float64 or totals.numel() < 4:
        raise CmlbmError(-1, "totals must be a device tensor of at least 4 float64")
    _check(load_library().cmlbm_step_totals(h, _ptr(f_in), _ptr(f_out), _ptr(totals), _stream(stream)), h)


def cmlbm_step_totals_noalloc(h, f_in, f_out, totals, stream=None):
    if totals.dtype != torch.float64 or totals.numel() < 4:
        raise CmlbmError(-1, "totals must be a device tensor of at least 4 float64")
    _check(load_library().cmlbm_step_totals_noalloc(h, _ptr(f_in), _ptr(f_out), _ptr(totals), _stream(stream)), h)


def cmlbm_run(h, f_a, f_b, nsteps, stream=None):
    flag = ctypes.c_int(0)
    _check(load_library().cmlbm_run(h, _ptr(f_a), _ptr(f_b), int(nsteps), _stream(stream), ctypes.byref(flag)), h)
    return bool(flag.value)


def cmlbm_gather_precollision(h, f_post, f_pre, stream=None):
    _check(load_library().cmlbm_gather_precollision(h, _ptr(f_post), _ptr(f_pre), _stream(stream)), h)


def cmlbm_export_populations(h, f_buf, f_soa, stream=None):
    _check(load_library().cmlbm_export_populations(h, _ptr(f_buf), _ptr(f_soa), _stream(stream)), h)


def cmlbm_import_populations(h, f_soa, f_buf, stream=None):
    _check(load_library().cmlbm_import_populations(h, _ptr(f_soa), _ptr(f_buf), _stream(stream)), h)


def cmlbm_macroscopic(h, f_post, rho, u, stream=None):
    _check(load_library().cmlbm_macroscopic(h, _ptr(f_post), _ptr(rho), _ptr(u), _stream(stream)), h)


def cmlbm_totals(h, f_post, stream=None):
    out = (ctypes.c_double * 4)()
    _check(load_library().cmlbm_totals(h, _ptr(f_post), out, _stream(stream)), h)
    return [out[i] for i in range(4)]


def cmlbm_init_equilibrium_inplace(h, rho, u, f, stream=None):
    _check(load_library().cmlbm_init_equilibrium_inplace(h, _ptr(rho), _ptr(u), _ptr(f), _stream(stream)), h)


def cmlbm_step_inplace(h, f, parity, stream=None):
    _check(load_library().cmlbm_step_inplace(h, _ptr(f), int(parity), _stream(stream)), h)


def cmlbm_step_inplace_totals(h, f, parity, totals, stream=None):
    if totals.dtype != torch.float64 or totals.numel() < 4:
        raise CmlbmError(-1, "totals must be a device tensor of at least 4 float64")
    _check(load_library().cmlbm_step_inplace_totals(h, _ptr(f), int(parity), _ptr(totals), _stream(stream)), h)


def cmlbm_run_inplace(h, f, nsteps, stream=None):
    _check(load_library().cmlbm_run_inplace(h, _ptr(f), int(nsteps), _stream(stream)), h)


def cmlbm_macroscopic_pre(h, f_pre_buf, rho, u, stream=None):
    _check(load_library().cmlbm_macroscopic_pre(h, _ptr(f_pre_buf), _ptr(rho), _ptr(u), _stream(stream)), h)


def cmlbm_totals_pre(h, f_pre_buf, stream=None):
    out = (ctypes.c_double * 4)()
    _check(load_library().cmlbm_totals_pre(h, _ptr(f_pre_buf), out, _stream(stream)), h)
    return [out[i] for i in range(4)]


def cmlbm_adjoint_step(h, f_post_prev, lam_next, lam, dLdF, dLdomega, stream=None):
    _check(load_library().cmlbm_adjoint_step(h, _ptr(f_post_prev), _ptr(lam_next), _ptr(lam), _ptr(dLdF),
                                              _ptr(dLdomega), _stream(stream)), h)


def cmlbm_wall_sensitivity(h, f_post_prev, lam_next, dLdphi, stream=None):
    _check(load_library().cmlbm_wall_sensitivity(h, _ptr(f_post_prev), _ptr(lam_next), _ptr(dLdphi),
                                                  _stream(stream)), h)


def cmlbm_wall_sensitivity_post(h, f_post, lam, dLdphi, stream=None):
    _check(load_library().cmlbm_wall_sensitivity_post(h, _ptr(f_post), _ptr(lam), _ptr(dLdphi), _stream(stream)), h)


def cmlbm_check_finite(h, f_buf, stream=None):
    out = ctypes.c_int64(0)
    _check(load_library().cmlbm_check_finite(h, _ptr(f_buf), ctypes.byref(out), _stream(stream)), h)
    return out.value


def cmlbm_kinetic_energy_sum(h, f_pre, stream=None):
    out = ctypes.c_double(0.0)
    _check(load_library().cmlbm_kinetic_energy_sum(h, _ptr(f_pre), ctypes.byref(out), _stream(stream)), h)
    return out.value


def cmlbm_kinetic_energy_seed(h, f_pre, scale, lam, dLdF, stream=None):
    _check(load_library().cmlbm_kinetic_energy_seed(h, _ptr(f_pre), float(scale), _ptr(lam), _ptr(dLdF),
                                                     _stream(stream)), h)


def cmlbm_init_adjoint(h, u0, lam0, dLdF, stream=None):
    _check(load_library().cmlbm_init_adjoint(h, _ptr(u0), _ptr(lam0), _ptr(dLdF), _stream(stream)), h)


def cmlbm_version():
    return load_library().cmlbm_version().decode()


# ----------------------------------------------------------------------------
# A handle with its buffers' shapes (still marshalling only)
# ----------------------------------------------------------------------------
class Sim:
    """Owns one cmlbm handle.  Shapes: populations (Q, nz, ny, nx), scalars
    (nz, ny, nx), vectors (3, nz, ny, nx).  The C calls take bare pointers, so
    every tensor passed here is checked first for device, dtype and size: a
    short buffer would otherwise be read or written past its end."""

    def __init__(self, q, nx, ny, nz, precision=F32, device=None):
        self.q, self.nx, self.ny, self.nz, self.precision = q, nx, ny, nz, precision
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        with torch.cuda.device(self.device):
            self.h = cmlbm_create(q, nx, ny, nz, precision)
        self.real = real_dtype(precision)
        self.store = storage_dtype(precision)
        self._keep = {}

    def close(self):
        if getattr(self, "h", None) is not None:
            cmlbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # buffers -----------------------------------------------------------
    @property
    def nodes(self):
        return self.nx * self.ny * self.nz

    def _need(self, t, dtype, numel, name):
        """Device, dtype and size check of a tensor argument (raw integer
        pointers pass unchecked)."""
        if isinstance(t, torch.Tensor):
            if t.device != self.device or t.dtype != dtype or t.numel() < numel:
                raise CmlbmError(-1, f"{name}: expected a {dtype} tensor of at least {numel} elements on "
                                     f"{self.device}, got {t.dtype}, {t.numel()} elements on {t.device}")
        return t

    def _pop(self, t, name):
        return self._need(t, self.store, self.q * self.nodes, name)

    def _realpop(self, t, name):
        return self._need(t, self.real, self.q * self.nodes, name)

    def _dLdF(self, t):
        return self._need(t, torch.float64, 3 * self.nodes if "force" in self._keep else 3, "dLdF")

    def populations(self):
        return torch.empty((self.q, self.nz, self.ny, self.nx), dtype=self.store, device=self.device)

    def real_populations(self):
        return torch.empty((self.q, self.nz, self.ny, self.nx), dtype=self.real, device=self.device)

    # settings ----------------------------------------------------------
    def set_rates(self, omega):
        cmlbm_set_rates(self.h, list(omega))

    def set_force(self, F):
        """F: 3 numbers (uniform) or a (3, nz, ny, nx) real tensor (field)."""
        if isinstance(F, torch.Tensor) and F.dim() == 4:
            F = F.to(device=self.device, dtype=self.real).contiguous()
            if F.numel() != 3 * self.nodes:
                raise CmlbmError(-1, f"force field: expected shape (3, {self.nz}, {self.ny}, {self.nx})")
            self._keep["force"] = F
            cmlbm_set_force_field(self.h, F)
        else:
            self._keep.pop("force", None)
            fx, fy, fz = [float(v) for v in F]
            cmlbm_set_force_uniform(self.h, fx, fy, fz)

    def set_force_scale(self, scale):
        cmlbm_set_force_scale(self.h, scale)

    def set_attractor_per_mass(self, per_mass=True):
        cmlbm_set_attractor_per_mass(self.h, per_mass)

    def set_mask(self, solid):
        if solid is None:
            self._keep.pop("mask", None)
            cmlbm_set_mask(self.h, None)
            return
        m = solid.to(device=self.device, dtype=torch.uint8).contiguous()
        if m.numel() != self.nodes:
            raise CmlbmError(-1, f"mask: expected shape ({self.nz}, {self.ny}, {self.nx})")
        self._keep["mask"] = m
        cmlbm_set_mask(self.h, m)

    # work --------------------------------------------------------------
    def init_equilibrium(self, rho, u, f_post=None, f_pre=None, stream=None):
        rho = rho.to(device=self.device, dtype=self.real).contiguous()
        u = u.to(device=self.device, dtype=self.real).contiguous()
        f_post = self.populations() if f_post is None else self._pop(f_post, "f_post")
        f_pre = self.real_populations() if f_pre is None else self._realpop(f_pre, "f_pre")
        self._need(rho, self.real, self.nodes, "rho")
        self._need(u, self.real, 3 * self.nodes, "u")
        cmlbm_init_equilibrium(self.h, rho, u, f_pre, f_post, stream)
        return f_post, f_pre

    def step(self, f_in, f_out, stream=None, totals=None):
        """One step f_in -> f_out.  With `totals` (4 float64 on the device), the
        same pass also writes the FP64 (mass, momentum) of f_in's state."""
        self._pop(f_in, "f_in")
        self._pop(f_out, "f_out")
        if totals is None:
            cmlbm_step(self.h, f_in, f_out, stream)
        else:
            cmlbm_step_totals(self.h, f_in, f_out, totals, stream)

    def run(self, f_a, f_b, nsteps, stream=None):
        """Returns the buffer holding the last state."""
        self._pop(f_a, "f_a")
        self._pop(f_b, "f_b")
        return f_b if cmlbm_run(self.h, f_a, f_b, nsteps, stream) else f_a

    def gather(self, f_post, out=None, stream=None):
        out = self.real_populations() if out is None else self._realpop(out, "out")
        cmlbm_gather_precollision(self.h, self._pop(f_post, "f_post"), out, stream)
        return out

    def export_populations(self, f_buf, out=None, stream=None):
        out = self.real_populations() if out is None else self._realpop(out, "out")
        cmlbm_export_populations(self.h, self._pop(f_buf, "f_buf"), out, stream)
        return out

    def import_populations(self, f_soa, f_buf=None, stream=None):
        f_buf = self.populations() if f_buf is None else self._pop(f_buf, "f_buf")
        f_soa = self._realpop(f_soa.to(device=self.device, dtype=self.real).contiguous(), "f_soa")
        cmlbm_import_populations(self.h, f_soa, f_buf, stream)
        return f_buf

    def macroscopic(self, f_post, stream=None):
        rho = torch.empty((self.nz, self.ny, self.nx), dtype=self.real, device=self.device)
        u = torch.empty((3, self.nz, self.ny, self.nx), dtype=self.real, device=self.device)
        cmlbm_macroscopic(self.h, self._pop(f_post, "f_post"), rho, u, stream)
        return rho, u

    def totals(self, f_post, stream=None):
        return cmlbm_totals(self.h, self._pop(f_post, "f_post"), stream)

    # in-place stepping (one buffer; phase 0 = pre-collision populations) --
    def init_equilibrium_inplace(self, rho, u, f=None, stream=None):
        """fbar(x, 0) into an in-place buffer (phase 0)."""
        rho = rho.to(device=self.device, dtype=self.real).contiguous()
        u = u.to(device=self.device, dtype=self.real).contiguous()
        f = self.populations() if f is None else self._pop(f, "f")
        self._need(rho, self.real, self.nodes, "rho")
        self._need(u, self.real, 3 * self.nodes, "u")
        cmlbm_init_equilibrium_inplace(self.h, rho, u, f, stream)
        return f

    def step_inplace(self, f, parity, stream=None, totals=None):
        """One in-place step; with `totals` (4 float64 on the device), the same
        pass also writes the FP64 (mass, momentum) of the state it collides."""
        self._pop(f, "f")
        if totals is None:
            cmlbm_step_inplace(self.h, f, parity, stream)
        else:
            cmlbm_step_inplace_totals(self.h, f, parity, totals, stream)

    def run_inplace(self, f, nsteps, stream=None):
        """nsteps (even) in-place steps; f holds the pre-collision state in
        phase 0 before and after."""
        cmlbm_run_inplace(self.h, self._pop(f, "f"), nsteps, stream)
        return f

    def macroscopic_pre(self, f_pre_buf, stream=None):
        rho = torch.empty((self.nz, self.ny, self.nx), dtype=self.real, device=self.device)
        u = torch.empty((3, self.nz, self.ny, self.nx), dtype=self.real, device=self.device)
        cmlbm_macroscopic_pre(self.h, self._pop(f_pre_buf, "f_pre_buf"), rho, u, stream)
        return rho, u

    def totals_pre(self, f_pre_buf, stream=None):
        return cmlbm_totals_pre(self.h, self._pop(f_pre_buf, "f_pre_buf"), stream)

    def adjoint_step(self, f_post_prev, lam_next, lam, dLdF, dLdomega, stream=None):
        self._pop(f_post_prev, "f_post_prev")
        self._realpop(lam_next, "lam_next")
        self._realpop(lam, "lam")
        self._dLdF(dLdF)
        self._need(dLdomega, torch.float64, self.q - 4, "dLdomega")
        cmlbm_adjoint_step(self.h, f_post_prev, lam_next, lam, dLdF, dLdomega, stream)

    def wall_sensitivity(self, f_post_prev, lam_next, dLdphi, stream=None):
        self._pop(f_post_prev, "f_post_prev")
        self._realpop(lam_next, "lam_next")
        self._need(dLdphi, torch.float64, self.nodes, "dLdphi")
        cmlbm_wall_sensitivity(self.h, f_post_prev, lam_next, dLdphi, stream)

    def wall_sensitivity_post(self, f_post, lam, dLdphi, stream=None):
        self._pop(f_post, "f_post")
        self._realpop(lam, "lam")
        self._need(dLdphi, torch.float64, self.nodes, "dLdphi")
        cmlbm_wall_sensitivity_post(self.h, f_post, lam, dLdphi, stream)

    def check_finite(self, f_buf, stream=None):
        """Number of NaN or +-Inf stored populations of fluid nodes in a
        population buffer (two-buffer or in-place, either phase)."""
        return cmlbm_check_finite(self.h, self._pop(f_buf, "f_buf"), stream)

    def kinetic_energy_sum(self, f_pre, stream=None):
        return cmlbm_kinetic_energy_sum(self.h, self._realpop(f_pre, "f_pre"), stream)

    def kinetic_energy_seed(self, f_pre, scale, lam, dLdF, stream=None):
        self._realpop(f_pre, "f_pre")
        self._realpop(lam, "lam")
        self._dLdF(dLdF)
        cmlbm_kinetic_energy_seed(self.h, f_pre, scale, lam, dLdF, stream)

    def init_adjoint(self, u0, lam0, dLdF, stream=None):
        self._need(u0, self.real, 3 * self.nodes, "u0")
        self._realpop(lam0, "lam0")
        self._dLdF(dLdF)
        cmlbm_init_adjoint(self.h, u0, lam0, dLdF, stream)
