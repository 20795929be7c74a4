"""Thin ctypes binding of librrt.so (C ABI in include/rrt.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  Host arrays are float64 NumPy arrays in the layouts of rrt.h (lab
intensities [K][P][G], boundaries [K][ny][nx][G]).  The
library must have been built (``__graft_entry__.build()``); loading fails
loudly otherwise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librrt.so")

RRT_OK, RRT_E_INVALID, RRT_E_HOST_OOM, RRT_E_HBM, RRT_E_NOT_CONVERGED, RRT_E_DEVICE, RRT_E_STATE = 0, -1, -2, -3, -4, -5, -6
FP64, FP32, MIXED = 0, 1, 2
THOMSON, COMPTON = 0, 1
FRAME_LAB, FRAME_COMOVING = 0, 1
SCHEME_RK4, SCHEME_EULER = 0, 1
STATUS_NAMES = {0: "RRT_OK", -1: "RRT_E_INVALID", -2: "RRT_E_HOST_OOM", -3: "RRT_E_HBM",
                -4: "RRT_E_NOT_CONVERGED", -5: "RRT_E_DEVICE", -6: "RRT_E_STATE"}

_dp = ctypes.POINTER(ctypes.c_double)


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double)]


class Groups(ctypes.Structure):
    _fields_ = [("ngroups", ctypes.c_int), ("edges", _dp), ("log_centres", ctypes.c_int), ("mec2", ctypes.c_double)]


class Angles(ctypes.Structure):
    _fields_ = [("lmax", ctypes.c_int), ("n_mu", ctypes.c_int), ("n_phi", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("updates", ctypes.c_longlong)]


class RRTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load librrt.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first (__graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        sigs = {
            "rrt_create": [ctypes.POINTER(Grid), ctypes.POINTER(Groups), ctypes.POINTER(Angles), I, I, P, ctypes.POINTER(P)],
            "rrt_set_medium": [P, _dp, _dp, _dp, _dp, _dp],
            "rrt_set_boundary": [P, I, _dp],
            "rrt_set_intensity": [P, _dp],
            "rrt_set_source_sh": [P, _dp],
            "rrt_sweep": [P, D, ctypes.POINTER(Info)],
            "rrt_solve": [P, D, I, I, ctypes.POINTER(Info)],
            "rrt_advance": [P, D, I, I, D, I, I, ctypes.POINTER(Info)],
            "rrt_get_moments": [P, I, _dp, _dp, _dp],
            "rrt_get_source_sh": [P, _dp],
            "rrt_get_intensity_sh": [P, _dp],
            "rrt_get_intensity": [P, _dp],
            "rrt_get_sweep_intensity": [P, _dp],
            "rrt_get_compton_tables": [P, ctypes.POINTER(I), _dp, _dp, _dp],
            "rrt_get_moments_integrated": [P, I, _dp],
            "rrt_compton_tables": [I, _dp, I, D, I, I, _dp, _dp, _dp, P],
            "rrt_ray_trace": [P, _dp, _dp, _dp],
            "rrt_get_lab_source": [P, D, _dp],
            "rrt_set_medium_dev": [P, P, P, P, P, P],
            "rrt_set_intensity_dev": [P, P],
            "rrt_set_source_sh_dev": [P, P],
            "rrt_get_source_sh_dev": [P, P],
            "rrt_get_intensity_sh_dev": [P, P],
            "rrt_get_intensity_dev": [P, P],
            "rrt_get_sweep_intensity_dev": [P, P],
            "rrt_get_lab_source_dev": [P, D, P],
            "rrt_get_moments_dev": [P, I, P, P, P],
            "rrt_get_moments_integrated_dev": [P, I, P],
            "rrt_ray_trace_dev": [P, P, P, P],
            "rrt_vet_step": [P, D, I, _dp, _dp, _dp, _dp, _dp, _dp],
            "rrt_vet_step_dev": [P, D, I, P, P, P, P, P, P],
            "rrt_set_profiling": [P, I],
            "rrt_set_graphs": [P, I],
            "rrt_set_autotune": [P, I],
            "rrt_set_variants": [P, I, I],
            "rrt_get_variants": [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)],
            "rrt_graph_count": [P, ctypes.POINTER(I)],
            "rrt_kernel_time": [P, ctypes.c_char_p, ctypes.POINTER(I), ctypes.POINTER(D)],
            "rrt_synchronize": [P],
            "rrt_batch_create": [ctypes.c_size_t, ctypes.POINTER(P)],
            "rrt_batch_admit": [P, P, D, I, I],
            "rrt_batch_step": [P, I, ctypes.POINTER(I)],
            "rrt_batch_poll": [P, P, ctypes.POINTER(I), ctypes.POINTER(Info)],
            "rrt_batch_remove": [P, P],
        }
        for name, args in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.rrt_destroy.argtypes = [P]
        L.rrt_destroy.restype = None
        L.rrt_last_error.argtypes = []
        L.rrt_last_error.restype = ctypes.c_char_p
        L.rrt_footprint_bytes.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Groups), ctypes.POINTER(Angles), I, I, I]
        L.rrt_footprint_bytes.restype = ctypes.c_size_t
        L.rrt_device_bytes.argtypes = [P]
        L.rrt_device_bytes.restype = ctypes.c_size_t
        L.rrt_set_device_pool.argtypes = [ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
        L.rrt_set_device_pool.restype = I
        L.rrt_batch_destroy.argtypes = [P]
        L.rrt_batch_destroy.restype = None
        _lib = L
    return _lib


def _check(status, allow=()):
    if status != RRT_OK and status not in allow:
        raise RRTError(status, lib().rrt_last_error().decode())
    return status


def _in(a):
    if a is None:
        return None, ctypes.cast(None, _dp)
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _structs(spec):
    edges = spec.get("edges")
    e_arr, e_ptr = _in(edges)
    G = 1 if edges is None else len(edges) - 1
    grid = Grid(spec["nx"], spec["ny"], spec["nz"], spec["lx"], spec["ly"], spec["lz"])
    groups = Groups(G, e_ptr, int(spec.get("log_centres", True)), float(spec.get("mec2", 510.99895)))
    angles = Angles(spec["lmax"], spec["nmu"], spec["nphi"])
    return grid, groups, angles, e_arr


def set_device_pool(max_bytes):
    """Keep up to max_bytes of the device memory destroyed problems free, for reuse
    by later problems of the same sizes (rrt_set_device_pool); 0 frees it all.
    Returns the bytes held."""
    held = ctypes.c_size_t(0)
    _check(lib().rrt_set_device_pool(int(max_bytes), ctypes.byref(held)))
    return held.value


def compton_tables(edges, mec2, lmax, kT, log_centres=True, stream=None):
    """Stand-alone Compton tables at the temperatures kT (units of the edges):
    s [nt][G] and p [nt][lmax+1][G][G] (built on the GPU)."""
    e, ep = _in(edges)
    t, tp = _in(np.atleast_1d(kT))
    G, nt = len(e) - 1, len(t)
    s = np.zeros((nt, G))
    p = np.zeros((nt, lmax + 1, G, G))
    _check(lib().rrt_compton_tables(G, ep, int(log_centres), float(mec2), int(lmax), nt, tp, s.ctypes.data_as(_dp),
                                    p.ctypes.data_as(_dp), ctypes.c_void_p(stream) if stream else None))
    return s, p


def footprint_bytes(spec, precision=FP32, time_dependent=False, use_ng=False):
    grid, groups, angles, keep = _structs(spec)
    return lib().rrt_footprint_bytes(ctypes.byref(grid), ctypes.byref(groups), ctypes.byref(angles),
                                     precision, int(time_dependent), int(use_ng))


class Problem:
    """One radiative-transfer problem on the device (see rrt.h for the physics)."""

    def __init__(self, spec, precision=FP32, stream=None):
        L = lib()
        self.spec = spec
        grid, groups, angles, self._edges = _structs(spec)
        self.nx, self.ny, self.nz = spec["nx"], spec["ny"], spec["nz"]
        self.P = self.nx * self.ny * self.nz
        self.G = groups.ngroups
        self.K = spec["nmu"] * spec["nphi"]
        self.NL = (spec["lmax"] + 1) ** 2
        self.precision = precision
        scatter = COMPTON if spec.get("scatter", "thomson") == "compton" else THOMSON
        h = ctypes.c_void_p()
        _check(L.rrt_create(ctypes.byref(grid), ctypes.byref(groups), ctypes.byref(angles), scatter, precision,
                            ctypes.c_void_p(stream) if stream else None, ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_spec(cls, spec, precision=FP32, stream=None):
        """Create a problem and upload its medium and boundaries from a workload dict."""
        pr = cls(spec, precision, stream)
        kte = spec.get("kte") if spec.get("scatter", "thomson") == "compton" else None
        pr.set_medium(spec["kappa"], spec["sigma"], spec["bnu"], spec.get("beta"), kte)
        if spec.get("bc_bot") is not None:
            pr.set_boundary(0, spec["bc_bot"])
        if spec.get("bc_top") is not None:
            pr.set_boundary(1, spec["bc_top"])
        return pr

    # shapes
    def lab_shape(self):
        return (self.K, self.P, self.G)

    def sh_shape(self):
        return (self.P, self.G, self.NL)

    def close(self):
        if getattr(self, "_h", None):
            lib().rrt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # inputs
    def set_medium(self, kappa, sigma, bnu, beta=None, kte=None):
        P, G = self.P, self.G
        k, kp = _in(np.broadcast_to(kappa, (P, G)))
        s, sp = _in(np.broadcast_to(sigma, (P,)))
        b, bp = _in(np.broadcast_to(bnu, (P, G)))
        v, vp = _in(beta)
        t, tp = _in(kte)
        _check(lib().rrt_set_medium(self._h, kp, sp, bp, vp, tp))

    def set_boundary(self, face, I_in):
        a, p = _in(I_in)
        _check(lib().rrt_set_boundary(self._h, face, p))

    def set_intensity(self, I_lab):
        a, p = _in(I_lab)
        _check(lib().rrt_set_intensity(self._h, p))

    def set_source_sh(self, S):
        a, p = _in(S)
        _check(lib().rrt_set_source_sh(self._h, p))

    # steps
    @staticmethod
    def _info(i):
        return {"iters": i.iters, "residual": i.residual, "seconds": i.seconds, "updates": i.updates}

    def sweep(self, dt_stage=0.0):
        i = Info()
        _check(lib().rrt_sweep(self._h, float(dt_stage), ctypes.byref(i)))
        return self._info(i)

    def solve(self, tol=1e-8, max_iter=200, use_ng=True, allow_not_converged=False):
        i = Info()
        st = _check(lib().rrt_solve(self._h, float(tol), int(max_iter), int(use_ng), ctypes.byref(i)),
                    allow=(RRT_E_NOT_CONVERGED,) if allow_not_converged else ())
        d = self._info(i)
        d["converged"] = st == RRT_OK
        return d

    def advance(self, dt, nsteps=1, scheme=SCHEME_RK4, tol=1e-8, max_iter=200, use_ng=False):
        i = Info()
        _check(lib().rrt_advance(self._h, float(dt), int(nsteps), int(scheme), float(tol), int(max_iter), int(use_ng),
                                 ctypes.byref(i)))
        return self._info(i)

    # outputs
    def moments(self, frame=FRAME_LAB):
        J = np.zeros((self.P, self.G))
        H = np.zeros((self.P, self.G, 3))
        K = np.zeros((self.P, self.G, 6))
        _check(lib().rrt_get_moments(self._h, frame, J.ctypes.data_as(_dp), H.ctypes.data_as(_dp), K.ctypes.data_as(_dp)))
        return J, H, K

    def moments_integrated(self, frame=FRAME_LAB):
        """Frequency-integrated J [P], H [P][3], K [P][6] and f = K/J [P][6]."""
        out = np.zeros((self.P, 16))
        _check(lib().rrt_get_moments_integrated(self._h, frame, out.ctypes.data_as(_dp)))
        return out[:, 0], out[:, 1:4], out[:, 4:10], out[:, 10:16]

    def _get(self, fn, shape):
        out = np.zeros(shape)
        _check(fn(self._h, out.ctypes.data_as(_dp)))
        return out

    def source_sh(self):
        return self._get(lib().rrt_get_source_sh, self.sh_shape())

    def intensity_sh(self):
        return self._get(lib().rrt_get_intensity_sh, self.sh_shape())

    def intensity(self):
        return self._get(lib().rrt_get_intensity, self.lab_shape())

    def sweep_intensity(self):
        return self._get(lib().rrt_get_sweep_intensity, self.lab_shape())

    def compton_tables(self):
        """(node temperatures [nt], s [nt][G], A [nt][lmax+1][G][G]) in use."""
        nt = ctypes.c_int(0)
        _check(lib().rrt_get_compton_tables(self._h, ctypes.byref(nt), None, None, None))
        n = nt.value
        nl = self.spec["lmax"] + 1
        kT, s, A = np.zeros(n), np.zeros((n, self.G)), np.zeros((n, nl, self.G, self.G))
        _check(lib().rrt_get_compton_tables(self._h, ctypes.byref(nt), kT.ctypes.data_as(_dp), s.ctypes.data_as(_dp),
                                            A.ctypes.data_as(_dp)))
        return kT, s, A

    def ray_trace(self, S_tilde, chi_tilde):
        s, sp = _in(S_tilde)
        x, xp = _in(chi_tilde)
        out = np.zeros(self.lab_shape())
        _check(lib().rrt_ray_trace(self._h, sp, xp, out.ctypes.data_as(_dp)))
        return out

    # kernel variants
    def lab_source(self, dt_stage=0.0):
        """S~ [K][P][G] that the next sweep(dt_stage) traces (S2 + S3 of the current source)."""
        out = np.zeros(self.lab_shape())
        _check(lib().rrt_get_lab_source(self._h, float(dt_stage), out.ctypes.data_as(_dp)))
        return out

    # device-pointer variants: torch tensors on the GPU, in the working precision
    # (float64 for FP64, float32 otherwise; the medium and moments in float64)
    def _dev(self, t, shape, fp64=None):
        import torch
        want = torch.float64 if (fp64 if fp64 is not None else self.precision == FP64) else torch.float32
        if not (t.is_cuda and t.dtype == want and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
            raise ValueError(f"need a contiguous {want} CUDA tensor of shape {tuple(shape)}")
        return ctypes.c_void_p(t.data_ptr())

    def _new_dev(self, shape, fp64=None):
        import torch
        dt = torch.float64 if (fp64 if fp64 is not None else self.precision == FP64) else torch.float32
        return torch.empty(shape, dtype=dt, device="cuda")

    def set_medium_dev(self, kappa, sigma, bnu, beta=None, kte=None):
        P, G = self.P, self.G
        args = [self._dev(kappa, (P, G), True), self._dev(sigma, (P,), True), self._dev(bnu, (P, G), True),
                self._dev(beta, (P, 3), True) if beta is not None else None,
                self._dev(kte, (P,), True) if kte is not None else None]
        _check(lib().rrt_set_medium_dev(self._h, *args))

    def set_intensity_dev(self, I_lab):
        _check(lib().rrt_set_intensity_dev(self._h, self._dev(I_lab, self.lab_shape())))

    def set_source_sh_dev(self, S):
        _check(lib().rrt_set_source_sh_dev(self._h, self._dev(S, self.sh_shape())))

    def _get_dev(self, fn, shape, *pre):
        out = self._new_dev(shape)
        _check(fn(self._h, *pre, self._dev(out, shape)))
        return out

    def source_sh_dev(self):
        return self._get_dev(lib().rrt_get_source_sh_dev, self.sh_shape())

    def intensity_sh_dev(self):
        return self._get_dev(lib().rrt_get_intensity_sh_dev, self.sh_shape())

    def intensity_dev(self):
        return self._get_dev(lib().rrt_get_intensity_dev, self.lab_shape())

    def sweep_intensity_dev(self):
        return self._get_dev(lib().rrt_get_sweep_intensity_dev, self.lab_shape())

    def lab_source_dev(self, dt_stage=0.0):
        return self._get_dev(lib().rrt_get_lab_source_dev, self.lab_shape(), ctypes.c_double(dt_stage))

    def moments_dev(self, frame=FRAME_LAB):
        J = self._new_dev((self.P, self.G), True)
        H = self._new_dev((self.P, self.G, 3), True)
        K = self._new_dev((self.P, self.G, 6), True)
        _check(lib().rrt_get_moments_dev(self._h, frame, self._dev(J, J.shape, True), self._dev(H, H.shape, True),
                                         self._dev(K, K.shape, True)))
        return J, H, K

    def moments_integrated_dev(self, frame=FRAME_LAB):
        out = self._new_dev((self.P, 16), True)
        _check(lib().rrt_get_moments_integrated_dev(self._h, frame, self._dev(out, out.shape, True)))
        return out

    def ray_trace_dev(self, S_tilde, chi_tilde):
        out = self._new_dev(self.lab_shape())
        _check(lib().rrt_ray_trace_dev(self._h, self._dev(S_tilde, self.lab_shape()), self._dev(chi_tilde, self.lab_shape()),
                                       self._dev(out, self.lab_shape())))
        return out

    # variable-Eddington-tensor hand-off
    def vet_step(self, dt, nsteps, kappa_E, chi_F, B, J, H):
        """nsteps steps of the moment equations closed with the state's Eddington
        tensor: returns (J [P], H [P][3], G [P][4])."""
        P = self.P
        k, kp = _in(np.broadcast_to(kappa_E, (P,)))
        c, cp = _in(np.broadcast_to(chi_F, (P,)))
        b, bp = _in(np.broadcast_to(B, (P,)))
        J = np.array(np.broadcast_to(J, (P,)), dtype=np.float64)
        H = np.array(np.broadcast_to(H, (P, 3)), dtype=np.float64)
        G = np.zeros((P, 4))
        _check(lib().rrt_vet_step(self._h, float(dt), int(nsteps), kp, cp, bp, J.ctypes.data_as(_dp),
                                  H.ctypes.data_as(_dp), G.ctypes.data_as(_dp)))
        return J, H, G

    def vet_step_dev(self, dt, nsteps, kappa_E, chi_F, B, J, H, G=None):
        """The same on float64 CUDA tensors, J and H (and G) updated in place."""
        P = self.P
        _check(lib().rrt_vet_step_dev(self._h, float(dt), int(nsteps), self._dev(kappa_E, (P,), True),
                                      self._dev(chi_F, (P,), True), self._dev(B, (P,), True),
                                      self._dev(J, (P,), True), self._dev(H, (P, 3), True),
                                      self._dev(G, (P, 4), True) if G is not None else None))

    def set_autotune(self, enable=True):
        _check(lib().rrt_set_autotune(self._h, int(enable)))

    def set_variants(self, trace_groups=0, s6=-1):
        """Fix the kernel variants (turns autotuning off): trace_groups groups per
        ray-trace workgroup (0 keeps the current; -1 one group on group-major
        planes, the lab arrays transposed around the trace), s6 the ordinate -> SH product
        (-1 the default for the shape, 0 the library product, 1/2/4 the
        matrix-core kernel with that many 16-row tiles per wave)."""
        _check(lib().rrt_set_variants(self._h, int(trace_groups), int(s6)))

    def variants(self):
        gc, s6, tuned = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().rrt_get_variants(self._h, ctypes.byref(gc), ctypes.byref(s6), ctypes.byref(tuned)))
        return {"trace_groups": gc.value, "s6": s6.value, "tuned": bool(tuned.value)}

    # captured sweeps
    def set_graphs(self, enable=True):
        _check(lib().rrt_set_graphs(self._h, int(enable)))

    def graph_count(self):
        n = ctypes.c_int()
        _check(lib().rrt_graph_count(self._h, ctypes.byref(n)))
        return n.value

    # timing
    def set_profiling(self, enable=True):
        _check(lib().rrt_set_profiling(self._h, int(enable)))

    def kernel_time(self, name):
        n = ctypes.c_int()
        ms = ctypes.c_double()
        _check(lib().rrt_kernel_time(self._h, name.encode(), ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def synchronize(self):
        _check(lib().rrt_synchronize(self._h))

    def device_bytes(self):
        return lib().rrt_device_bytes(self._h)


class Batch:
    """Steady-state solves of independent problems sharing the GPU (rrt_batch_*):
    admission against a device-memory budget, rounds of one iteration per running
    solve, polling and removal.  The batch does not own its problems."""

    def __init__(self, max_hbm_bytes):
        h = ctypes.c_void_p()
        _check(lib().rrt_batch_create(int(max_hbm_bytes), ctypes.byref(h)))
        self._h = h

    def admit(self, problem, tol=1e-6, max_iter=200, use_ng=True):
        """True when admitted, False when the budget has no room."""
        st = lib().rrt_batch_admit(self._h, problem._h, float(tol), int(max_iter), int(use_ng))
        if st == RRT_E_HBM:
            return False
        _check(st)
        return True

    def step(self, rounds=1):
        n = ctypes.c_int()
        _check(lib().rrt_batch_step(self._h, int(rounds), ctypes.byref(n)))
        return n.value

    def poll(self, problem):
        """(done, info dict with "converged" once done)."""
        d = ctypes.c_int()
        i = Info()
        st = _check(lib().rrt_batch_poll(self._h, problem._h, ctypes.byref(d), ctypes.byref(i)),
                    allow=(RRT_E_NOT_CONVERGED,))
        info = Problem._info(i)
        if d.value:
            info["converged"] = st == RRT_OK
        return bool(d.value), info

    def remove(self, problem):
        _check(lib().rrt_batch_remove(self._h, problem._h))

    def close(self):
        if self._h:
            lib().rrt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
