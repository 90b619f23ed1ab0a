"""MI355X-native DDA solver: Python binding of the C ABI in include/dda.h.

Every step of the computation runs in libdda.so (HIP kernels for gfx950 and
its host code); this module only marshals arguments.  PyTorch supplies device
memory and streams.  If the library is missing, importing the API raises.

Typical use::

    import paper_1305_6497_amd as dda
    sites, box = dda.make_sites("ELLIPSOID", (20, 20, 20))
    kd = dda.kd_from_x(1.0, len(sites))
    t = dda.Target(sites, box, m=1.33 + 0.01j, kd=kd)
    rhs = [dda.orient_rhs(0, 0, 0, which=1), dda.orient_rhs(0, 0, 0, which=2)]
    P, stats = t.solve(rhs, tol=1e-5)
    q = t.cross_sections(rhs, P)
"""

import ctypes

import numpy as np

from . import _lib as L
from ._lib import DDAError  # noqa: F401

SHAPES = {"ELLIPSOID": L.DDA_SHAPE_ELLIPSOID, "RCTGLPRSM": L.DDA_SHAPE_RCTGLPRSM,
          "CYLINDER1": L.DDA_SHAPE_CYLINDER1, "HEX_PRISM": L.DDA_SHAPE_HEX_PRISM}
ALPHA = {"LATTDR": L.DDA_ALPHA_LDR, "LDR": L.DDA_ALPHA_LDR, "GKDLDR": L.DDA_ALPHA_GKDLDR, "CMRR": L.DDA_ALPHA_CMRR,
         "FLTRCD": L.DDA_ALPHA_FCD, "FCD": L.DDA_ALPHA_FCD}
SOLVER = {"bicgstab": 0, "bicgstab2": 1, "cocg": 2, "qmr": 3}
PRECISION = {"fp64": L.DDA_FP64, "mixed": L.DDA_MIXED, "mixed32": L.DDA_MIXED_V32}


def make_sites(shape, shpar):
    """Sites of a built-in shape: (int32 [N, 3] array, (nx, ny, nz))."""
    lib = L.lib()
    sp = (ctypes.c_double * 3)(*[float(v) for v in (tuple(shpar) + (1.0, 1.0, 1.0))[:3]])
    n = ctypes.c_int64()
    box = (ctypes.c_int32 * 3)()
    L.check(lib.dda_make_sites(SHAPES[shape], sp, ctypes.byref(n), box, None, 0))
    out = np.empty((n.value, 3), dtype=np.int32)
    L.check(lib.dda_make_sites(SHAPES[shape], sp, ctypes.byref(n), box,
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n.value))
    return out, tuple(box)


def aeff(n_sites):
    return L.lib().dda_aeff(int(n_sites))


def kd_from_x(x, n_sites):
    return L.lib().dda_kd_from_x(float(x), int(n_sites))


def next_smooth(n):
    return int(L.lib().dda_next_smooth(int(n)))


def orient_rhs(beta, theta, phi, e01=(0.0, 1.0, 0.0), which=1):
    """(khat, e) in the Target Frame for orientation (beta, theta, phi)."""
    e = (L.C64 * 3)(*[L.C64(complex(v).real, complex(v).imag) for v in e01])
    out = L.Rhs()
    L.check(L.lib().dda_orient_rhs(float(beta), float(theta), float(phi), e, int(which), ctypes.byref(out)))
    khat = np.array(list(out.khat))
    ev = np.array([complex(out.e[a].re, out.e[a].im) for a in range(3)])
    return khat, ev


def orientation_grid(beta=(0.0, 0.0, 1), theta=(0.0, 0.0, 1), phi=(0.0, 0.0, 1)):
    """Orientations (beta, theta, phi) in radians and weights of §20, each a
    (min, max, count) range; returns four float64 arrays of length
    nbeta * ntheta * nphi (beta fastest)."""
    n = int(beta[2]) * int(theta[2]) * int(phi[2])
    out = [np.empty(max(n, 1)) for _ in range(4)]
    ptr = [o.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for o in out]
    L.check(L.lib().dda_orientation_grid(float(beta[0]), float(beta[1]), int(beta[2]), float(theta[0]),
                                         float(theta[1]), int(theta[2]), float(phi[0]), float(phi[1]),
                                         int(phi[2]), *ptr))
    return tuple(o[:n] for o in out)


def _rhs_array(rhs):
    arr = (L.Rhs * len(rhs))()
    for i, (khat, e) in enumerate(rhs):
        for a in range(3):
            arr[i].khat[a] = float(khat[a])
            c = complex(e[a])
            arr[i].e[a] = L.C64(c.real, c.imag)
    return arr


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def fft_pencils(x, sign=-1, scale=1.0, stream=None):
    """Batched 1-D FFT of the last axis of a contiguous complex CUDA tensor."""
    import torch
    assert x.is_cuda and x.is_contiguous()
    prec = L.DDA_FP64 if x.dtype == torch.complex128 else L.DDA_MIXED
    assert x.dtype in (torch.complex128, torch.complex64)
    out = torch.empty_like(x)
    n = x.shape[-1]
    batch = x.numel() // n if n else 0
    L.check(L.lib().dda_fft_pencils(n, batch, int(sign), prec, float(scale), ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream), x.device.index or 0))
    return out


PASSES = {"x_forward": 0, "z_pass": 2, "x_inverse": 4}


def pass_plan(pass_name, length, precision="mixed", variant=0):
    """Radices (execution order) of plan `variant` of a pass ("x_forward",
    "z_pass" or "x_inverse") for a padded length."""
    r = (ctypes.c_int32 * 8)()
    n = L.check(L.lib().dda_pass_plan(PASSES[pass_name], int(length), PRECISION[precision], int(variant), r),
                ok=tuple(range(9)))
    return [r[i] for i in range(n)]


def zpass_plan(length, precision="mixed", variant=0):
    """Radices (execution order) of z-pass plan `variant` for a padded length."""
    return pass_plan("z_pass", length, precision, variant)


def footprint_bytes(box, n_sites, m=1.5, kd=0.5, nrhs=1, alpha="LATTDR"):
    """Device bytes a target and a solve of nrhs right-hand sides would hold."""
    mlist = m if isinstance(m, (list, tuple)) else [m]
    marr = (L.C64 * len(mlist))(*[L.C64(complex(v).real, complex(v).imag) for v in mlist])
    d = L.TargetDesc(nx=box[0], ny=box[1], nz=box[2], n_sites=int(n_sites), ijk=None, comp=None,
                     n_comp=len(mlist), m=marr, kd=float(kd), alpha_kind=ALPHA[alpha], device=0)
    out = ctypes.c_uint64()
    L.check(L.lib().dda_footprint_bytes(ctypes.byref(d), int(nrhs), None, ctypes.byref(out)))
    return out.value


def _checked_vec(v, nrhs, n, device=None):
    """A device vector argument: a contiguous complex128 CUDA tensor [nrhs, n, 3]
    (on cuda:device when given).  Raises ValueError naming what is wrong, before
    any pointer reaches the library."""
    import torch
    if not isinstance(v, torch.Tensor):
        raise ValueError(f"expected a torch tensor, got {type(v).__name__}")
    if v.dtype != torch.complex128:
        raise ValueError(f"expected dtype complex128, got {v.dtype}")
    if tuple(v.shape) != (nrhs, n, 3):
        raise ValueError(f"expected shape ({nrhs}, {n}, 3), got {tuple(v.shape)}")
    if not v.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if not v.is_cuda:
        raise ValueError("expected a CUDA (device) tensor, got a host tensor")
    if device is not None and (v.device.index or 0) != device:
        raise ValueError(f"expected a tensor on cuda:{device}, got {v.device}")
    return v


class Target:
    """A target handle: sites, refractive indices and wavenumber on one GPU."""

    def __init__(self, sites, box, m, kd, alpha="LATTDR", comp=None, device=0):
        self._lib = L.lib()
        self.sites = np.ascontiguousarray(sites, dtype=np.int32)
        self.n = self.sites.shape[0]
        mlist = list(m) if isinstance(m, (list, tuple, np.ndarray)) else [m]
        self._m = (L.C64 * len(mlist))(*[L.C64(complex(v).real, complex(v).imag) for v in mlist])
        self._comp = None if comp is None else np.ascontiguousarray(comp, dtype=np.uint8)
        self.device = device
        d = L.TargetDesc(nx=int(box[0]), ny=int(box[1]), nz=int(box[2]), n_sites=self.n,
                         ijk=self.sites.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         comp=None if self._comp is None else self._comp.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                         n_comp=len(mlist), m=self._m, kd=float(kd), alpha_kind=ALPHA[alpha], device=device)
        h = ctypes.c_void_p()
        self.setup_status = L.check(self._lib.dda_setup_target(ctypes.byref(d), ctypes.byref(h)),
                                    ok=(L.DDA_OK, L.DDA_WVALIDITY))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dda_free_target(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        i = L.TargetInfo()
        L.check(self._lib.dda_target_get_info(self._h, ctypes.byref(i)))
        return dict(box=tuple(i.box), grid=tuple(i.grid), n_sites=i.n_sites, kd=i.kd, aeff=i.aeff,
                    device_bytes=i.device_bytes,
                    plan_variant={name: dict(mixed=arr[0], fp64=arr[1]) for name, arr in
                                  (("x_forward", i.xfwd_variant), ("z_pass", i.zpass_variant),
                                   ("x_inverse", i.xinv_variant))})

    def set_plan_variant(self, pass_name, variant):
        """Force the radix-plan variant of "x_forward", "z_pass" or "x_inverse",
        or -1 for the tuned table's."""
        L.check(self._lib.dda_set_plan_variant(self._h, PASSES[pass_name], int(variant)))

    def set_zpass_variant(self, variant):
        """Force the z-pass radix-plan variant (0..3), or -1 for the tuned table's."""
        self.set_plan_variant("z_pass", variant)

    def _vec(self, nrhs):
        import torch
        return torch.empty((nrhs, self.n, 3), dtype=torch.complex128, device=f"cuda:{self.device}")

    def _checked(self, v, nrhs):
        """A device vector argument: contiguous complex128 [nrhs, N, 3] on this target's device."""
        return _checked_vec(v, nrhs, self.n, self.device)

    def solve(self, rhs, tol=1e-5, max_iter=1000, precision="fp64", inner_tol=0.0, max_outer=20, check_every=0,
              out=None, stream=None, use_graph=False, solver="bicgstab", fold_records=0, x0=None, jacobi=False):
        """Solve A P = E for every (khat, e) in rhs.  Returns (P, stats).

        solver: "bicgstab" (the guide's PBCGST), "bicgstab2" (BiCGstab(2), the
        guide's PBCGS2), "cocg" or "qmr" (QMR smoothing of COCG, the guide's
        QMRCCG).  check_every: iterations between host convergence checks; 0
        picks them from the residual decay after a first block of 8, -n does
        the same after a first block of n.  fold_records: tuning only (results
        are bit-identical), see dda_solve_opts.  x0: optional initial guess,
        a contiguous complex128 [nrhs, N, 3] device tensor (default P = 0).
        precision: "fp64", "mixed" (FP32 products, FP64 vectors) or "mixed32"
        (COCG and BiCGSTAB: also the search direction p and A p stored in FP32).
        jacobi: symmetric diagonal scaling S A S with S = diag(alpha)^(1/2)
        (tol then bounds |S(E - A P)| / |S E|, the same as |E - A P| / |E| for
        one composition with a scalar polarizability)."""
        nrhs = len(rhs)
        x0 = None if x0 is None else self._checked(x0, nrhs)
        P = self._vec(nrhs) if out is None else self._checked(out, nrhs)
        opts = L.SolveOpts(tol=tol, max_iter=max_iter, precision=PRECISION[precision], inner_tol=inner_tol,
                           max_outer=max_outer, check_every=check_every, use_graph=int(bool(use_graph)),
                           solver=SOLVER[solver], fold_records=fold_records,
                           x0=None if x0 is None else x0.data_ptr(), jacobi=int(bool(jacobi)))
        st = (L.SolveStats * nrhs)()
        code = L.check(self._lib.dda_solve(self._h, _rhs_array(rhs), nrhs, ctypes.byref(opts),
                                           ctypes.c_void_p(P.data_ptr()), None, _stream_ptr(stream), st),
                       ok=(L.DDA_OK, L.DDA_NOT_CONVERGED))
        stats = [dict(status=s.status, iters=s.iters, matvecs=s.matvecs, outer=s.outer, rel_resid=s.rel_resid)
                 for s in st]
        return P, stats

    def cross_sections(self, rhs, P, stream=None):
        nrhs = len(rhs)
        P = self._checked(P, nrhs)
        q = (L.Q * nrhs)()
        L.check(self._lib.dda_cross_sections(self._h, _rhs_array(rhs), nrhs, ctypes.c_void_p(P.data_ptr()), None,
                                             _stream_ptr(stream), q))
        return [dict(qext=v.qext, qabs=v.qabs, qsca=v.qsca, aeff=v.aeff, qpha=v.qpha) for v in q]

    def far_field(self, rhs, P, etasca=0.5, stream=None):
        """Q_sca by far-field quadrature, <cos theta>, <cos^2 theta> and Q_bk per RHS."""
        nrhs = len(rhs)
        P = self._checked(P, nrhs)
        out = (L.Far * nrhs)()
        L.check(self._lib.dda_far_field(self._h, _rhs_array(rhs), nrhs, ctypes.c_void_p(P.data_ptr()),
                                        float(etasca), _stream_ptr(stream), out))
        return [dict(qsca=v.qsca, g=v.g, cos2=v.cos2, n_theta=v.n_theta, n_phi=v.n_phi, qbk=v.qbk) for v in out]

    def scattering_matrix(self, rhs, P, lab, theta_phi, stream=None):
        """Amplitude and Mueller matrices for the two polarizations rhs[0], rhs[1]
        of one incidence: (f [ndir, 2, 2], S [ndir, 4], mueller [ndir, 4, 4])
        as NumPy arrays; lab = (x_LF, y_LF, z_LF) in the target frame,
        theta_phi [ndir, 2] in radians."""
        import numpy as np
        if len(rhs) != 2:
            raise ValueError("scattering_matrix takes the two polarizations of one incidence")
        P = self._checked(P, 2)
        tp = np.ascontiguousarray(theta_phi, dtype=np.float64).reshape(-1, 2)
        lb = np.ascontiguousarray(lab, dtype=np.float64).reshape(9)
        out = (L.Scat * len(tp))()
        L.check(self._lib.dda_scattering_matrix(
            self._h, _rhs_array(rhs), ctypes.c_void_p(P.data_ptr()),
            lb.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(tp),
            tp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream_ptr(stream), out))
        f = np.array([[[complex(o.f[m][l].re, o.f[m][l].im) for l in range(2)] for m in range(2)] for o in out])
        S = np.array([[complex(o.s[j].re, o.s[j].im) for j in range(4)] for o in out])
        M = np.array([[list(o.mueller[i]) for i in range(4)] for o in out])
        return f, S, M

    def near_field(self, rhs, P, margin=(0, 0, 0), macroscopic=False, magnetic=False, stream=None):
        """E at every lattice point of the box extended by ``margin`` points on
        both sides of each axis: complex128 [nrhs, Z, Y, X, 3] on the device,
        point (i, j, k) at site coordinate (i, j, k) - margin.  With
        magnetic=True returns (E, B), B the magnetic field at the same points."""
        import torch
        P = self._checked(P, len(rhs))
        mg = [int(v) for v in margin]
        box = self.info()["box"]
        X, Y, Z = (box[a] + 2 * mg[a] for a in range(3))
        out = torch.empty((len(rhs), Z, Y, X, 3), dtype=torch.complex128, device=f"cuda:{self.device}")
        if not magnetic:
            L.check(self._lib.dda_near_field(self._h, _rhs_array(rhs), len(rhs), ctypes.c_void_p(P.data_ptr()),
                                             (ctypes.c_int32 * 3)(*mg), int(bool(macroscopic)),
                                             ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
            return out
        outb = torch.empty_like(out)
        L.check(self._lib.dda_near_field_eb(self._h, _rhs_array(rhs), len(rhs), ctypes.c_void_p(P.data_ptr()),
                                            (ctypes.c_int32 * 3)(*mg), int(bool(macroscopic)),
                                            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(outb.data_ptr()),
                                            _stream_ptr(stream)))
        return out, outb

    def apply(self, rhs, P, precision="fp64", stream=None):
        nrhs = len(rhs)
        P = self._checked(P, nrhs)
        out = self._vec(nrhs)
        L.check(self._lib.dda_apply(self._h, _rhs_array(rhs), nrhs, PRECISION[precision],
                                    ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    _stream_ptr(stream)))
        return out

    def apply_noalloc(self, rhs, P, out, precision="fp64", stream=None):
        """A P into the caller's ``out`` through dda_apply_noalloc: the library
        allocates nothing (its work buffers are a static device array)."""
        nrhs = len(rhs)
        P = self._checked(P, nrhs)
        out = self._checked(out, nrhs)
        L.check(self._lib.dda_apply_noalloc(self._h, _rhs_array(rhs), nrhs, PRECISION[precision],
                                            ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                            _stream_ptr(stream)))
        return out

    def set_pass_timing(self, every=1):
        """Time the FFT passes of every `every`-th product inside solve() with HIP events (0: off);
        resets the sums."""
        L.check(self._lib.dda_set_pass_timing(self._h, int(every)))

    def pass_timing(self, precision="mixed"):
        """Average ms per launch of each pass over the products timed inside solves since
        set_pass_timing, and their count."""
        ms = (ctypes.c_double * 5)()
        n = ctypes.c_int64()
        L.check(self._lib.dda_get_pass_timing(self._h, PRECISION[precision], ms, ctypes.byref(n)))
        names = ("x_forward", "y_forward", "z_pass", "y_inverse", "x_inverse")
        avg = {k: (v / n.value if n.value else None) for k, v in zip(names, list(ms))}
        avg["total"] = sum(ms) / n.value if n.value else None
        return avg, n.value

    def profile_matvec(self, rhs, P, precision="mixed", reps=20, stream=None):
        """Average ms of each FFT pass (and the whole product) over reps products."""
        P = self._checked(P, len(rhs))
        out = self._vec(len(rhs))
        ms = (ctypes.c_double * 6)()
        L.check(self._lib.dda_profile_matvec(self._h, _rhs_array(rhs), len(rhs), PRECISION[precision], int(reps),
                                             ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                             _stream_ptr(stream), ms))
        names = ("x_forward", "y_forward", "z_pass", "y_inverse", "x_inverse", "total")
        return dict(zip(names, list(ms)))

    def incident_field(self, rhs, stream=None):
        out = self._vec(len(rhs))
        L.check(self._lib.dda_incident_field(self._h, _rhs_array(rhs), len(rhs), ctypes.c_void_p(out.data_ptr()),
                                             _stream_ptr(stream)))
        return out
