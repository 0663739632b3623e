"""ctypes binding of liblcmd.so (the C ABI in include/lcmd.h).

Argument marshalling only: every step of the computation runs in the library's HIP kernels.
PyTorch provides device memory (the caller-owned state buffer, the field workspace) and the
HIP stream.  Loading fails loudly if the library has not been built.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblcmd.so")

LC_MAX_Z = 16
LC_REC = 48
LC_DET_BINS = 120
LC_DET_SLOTS = LC_DET_BINS + 2

LC_OK, LC_E_INVALID, LC_E_CAPACITY, LC_E_NONFINITE, LC_E_HIP, LC_E_STATE, LC_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
PRECISIONS = {"fp64": 0, "fp32_acc64": 1, "fp32_kahan": 2}
ENVELOPES = {"gauss_field": 0, "gauss_intensity": 1, "sin2": 2, "flat": 3}
PHASES = {"dipole": 0, "plane_wave": 1}
POLARIZATIONS = {"linear_x": 0, "circular": 1}
BOUNDARIES = {"open": 0, "periodic": 1, "mixed": 2}
OFI = {"laser_only": 0, "local": 1}

# record columns (see include/lcmd.h)
R_T, R_STEP, R_N, R_NION, R_NEL = 0, 1, 2, 3, 4
R_KE_HALF, R_KE_BAR, R_PE, R_WL, R_WC, R_WSP = 5, 6, 7, 8, 9, 10
R_P, R_F, R_FABS, R_MEANZ, R_ABS_EV, R_DROPPED, R_EVENTS, R_ENV, R_KE_START = 11, 14, 17, 18, 19, 20, 21, 22, 23
R_ZHIST = 24


class LcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblcmd error {code}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("precision", ctypes.c_int32), ("ionize", ctypes.c_int32),
        ("ofi_field", ctypes.c_int32), ("lambda_um", ctypes.c_double), ("dt", ctypes.c_double),
        ("t0", ctypes.c_double), ("softening_nm", ctypes.c_double), ("diag_every", ctypes.c_int32),
        ("max_records", ctypes.c_int32), ("max_splits", ctypes.c_int32), ("max_pair_blocks", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("detector_r0", ctypes.c_double), ("detector_half_angle_deg", ctypes.c_double),
        ("boundary", ctypes.c_int32), ("collisional", ctypes.c_int32), ("box_r0", ctypes.c_double),
        ("t_switch", ctypes.c_double),
    ]


class ClusterDesc(ctypes.Structure):
    _fields_ = [
        ("r0_nm", ctypes.c_double), ("rw_angstrom", ctypes.c_double), ("mass_u", ctypes.c_double),
        ("ip_ev", ctypes.c_double * LC_MAX_Z), ("intensity_wcm2", ctypes.c_double),
        ("envelope", ctypes.c_int32), ("phase", ctypes.c_int32), ("fwhm_fs", ctypes.c_double),
        ("n_cycles", ctypes.c_double), ("n_ion", ctypes.c_int64), ("capacity", ctypes.c_int64),
        ("weight", ctypes.c_double), ("z_max", ctypes.c_int32), ("polarization", ctypes.c_int32),
        ("electron_offset_nm", ctypes.c_double), ("n_steps", ctypes.c_int64),
        ("lotz_q", ctypes.c_double * LC_MAX_Z), ("lotz_a", ctypes.c_double),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [
        ("targets_per_lane", ctypes.c_int32), ("waves_per_target", ctypes.c_int32),
        ("tile_sources", ctypes.c_int32), ("j_splits", ctypes.c_int32), ("persistent", ctypes.c_int32),
        ("scalar_sources", ctypes.c_int32), ("newton3", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {"R": self.targets_per_lane, "WJ": self.waves_per_target, "T": self.tile_sources,
                "S": self.j_splits, "persistent": self.persistent, "scalar": self.scalar_sources,
                "newton3": self.newton3}


def make_tuning(R=0, WJ=0, T=0, S=0, persistent=0, scalar=0, newton3=0):
    t = Tuning()
    t.targets_per_lane, t.waves_per_target, t.tile_sources, t.j_splits, t.persistent = R, WJ, T, S, persistent
    t.scalar_sources = scalar
    t.newton3 = newton3
    return t


def pair_blocks_for(capacities, block=128):
    """Rows per block the pair-once kernel needs for clusters of these capacities with blocks of
    at least `block` slots (pass as max_pair_blocks)."""
    return max(-(-int(c) // block) for c in capacities)


_lib = None


def lib():
    """Load liblcmd.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1307_3711_amd/build.py "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, i8p, i32p, i64p = (ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int8),
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64))
    cfgp, clp, tp = ctypes.POINTER(Config), ctypes.POINTER(ClusterDesc), ctypes.POINTER(Tuning)
    sig = {
        "lc_version": ([], ctypes.c_int),
        "lc_error_string": ([ctypes.c_int], ctypes.c_char_p),
        "lc_last_error": ([vp], ctypes.c_char_p),
        "lc_units": ([ctypes.c_double, ctypes.c_double, dp], ctypes.c_int),
        "lc_state_bytes": ([cfgp, clp, ctypes.c_int32], ctypes.c_size_t),
        "lc_create": ([ctypes.POINTER(vp), cfgp, clp, ctypes.c_int32, vp, ctypes.c_size_t, vp], ctypes.c_int),
        "lc_init_from_host": ([vp, ctypes.c_int32, ctypes.c_int64, dp, dp, i8p], ctypes.c_int),
        "lc_init_generate": ([vp, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
        "lc_start": ([vp], ctypes.c_int),
        "lc_pair_rows_fit": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, i64p],
                             ctypes.c_int),
        "lc_step": ([vp, ctypes.c_int64], ctypes.c_int),
        "lc_set_graph": ([vp, ctypes.c_int32], ctypes.c_int),
        "lc_read_diagnostics": ([vp, ctypes.c_int32, dp, ctypes.c_int32, i32p], ctypes.c_int),
        "lc_read_particles": ([vp, ctypes.c_int32, dp, dp, i8p, dp, dp, ctypes.c_int64, i64p], ctypes.c_int),
        "lc_read_field": ([vp, ctypes.c_int32, dp, ctypes.c_int64, i64p], ctypes.c_int),
        "lc_read_iedf": ([vp, ctypes.c_int32, i64p, dp], ctypes.c_int),
        "lc_step_index": ([vp], ctypes.c_int64),
        "lc_cluster_counters": ([vp, ctypes.c_int32, dp], ctypes.c_int),
        "lc_time_particle_kernels": ([vp, ctypes.c_int32, dp], ctypes.c_int),
        "lc_set_tuning": ([vp, tp], ctypes.c_int),
        "lc_get_tuning": ([vp, tp], ctypes.c_int),
        "lc_autotune": ([vp, ctypes.c_char_p, tp], ctypes.c_int),
        "lc_save_state": ([vp, ctypes.c_char_p], ctypes.c_int),
        "lc_load_state": ([vp, ctypes.c_char_p], ctypes.c_int),
        "lc_destroy": ([vp], None),
        "lc_profile_steps": ([vp, ctypes.c_int64, dp, i64p], ctypes.c_int),
        "lc_mlp_state_bytes": ([], ctypes.c_size_t),
        "lc_mlp_n_params": ([], ctypes.c_int),
        "lc_mlp_set_params": ([vp, vp, vp], ctypes.c_int),
        "lc_mlp_get_params": ([vp, vp, vp, vp], ctypes.c_int),
        "lc_mlp_fit_scaler": ([vp, vp, vp, ctypes.c_int64, vp], ctypes.c_int),
        "lc_mlp_train": ([vp, vp, vp, ctypes.c_int64, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, vp, vp],
                         ctypes.c_int),
        "lc_mlp_grad": ([vp, vp, vp, ctypes.c_int64, vp, ctypes.c_int32, vp, vp, vp], ctypes.c_int),
        "lc_mlp_infer": ([vp, vp, vp, ctypes.c_int64, vp], ctypes.c_int),
        "lc_mlp_status": ([vp, vp], ctypes.c_int),
        "lc_field_workspace_bytes": ([ctypes.c_int32, ctypes.c_int64, tp], ctypes.c_size_t),
        "lc_field": ([ctypes.c_int32, ctypes.c_int64, vp, ctypes.c_double, vp, vp, vp, ctypes.c_size_t, tp, vp],
                     ctypes.c_int),
        "lc_field_static": ([ctypes.c_int32, ctypes.c_int64, vp, ctypes.c_double, vp, vp, tp, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(code, handle=None):
    if code != LC_OK:
        L = lib()
        msg = L.lc_last_error(handle).decode() if handle else L.lc_error_string(code).decode()
        raise LcError(code, msg or L.lc_error_string(code).decode())


def units(lambda_um, intensity_wcm2=0.0):
    """The library's unit constants: kappa, field a.u. per a0, rate scale, a0, k (1/nm), m_e c^2 (eV)."""
    out = (ctypes.c_double * 6)()
    _check(lib().lc_units(float(lambda_um), float(intensity_wcm2), out))
    return {"kappa": out[0], "field_au": out[1], "rate_scale": out[2], "a0": out[3], "k_per_nm": out[4],
            "mec2_ev": out[5]}


def make_config(precision="fp64", ionize=True, ofi_field="laser_only", lambda_um=0.8, dt=0.05, t0=0.0,
                softening_nm=0.1, diag_every=10, max_records=1024, max_splits=32, seed=0, max_pair_blocks=0,
                detector_r0=0.0, detector_half_angle_deg=30.0, boundary="open", box_r0=20.0, t_switch=float("inf"),
                collisional=False):
    c = Config()
    c.struct_size = ctypes.sizeof(Config)
    c.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    c.ionize = 1 if ionize else 0
    c.ofi_field = OFI[ofi_field]
    c.lambda_um, c.dt, c.t0, c.softening_nm = lambda_um, dt, t0, softening_nm
    c.diag_every, c.max_records, c.max_splits, c.seed = diag_every, max_records, max_splits, seed
    c.max_pair_blocks = max_pair_blocks
    c.detector_r0, c.detector_half_angle_deg = detector_r0, detector_half_angle_deg
    c.boundary, c.box_r0, c.t_switch = BOUNDARIES[boundary], box_r0, t_switch
    c.collisional = 1 if collisional else 0
    return c


def make_cluster(species, r0_nm, n_ion, capacity, intensity_wcm2, envelope="gauss_field", fwhm_fs=30.0,
                 n_cycles=10.0, phase="dipole", weight=0.0, z_max=8, electron_offset_nm=0.01, n_steps=0,
                 polarization="linear_x", lotz_a=4.5e-14):
    """species: mapping with rw_angstrom, mass_u and ip_ev (charge state k -> k+1, eV)."""
    d = ClusterDesc()
    d.r0_nm, d.rw_angstrom, d.mass_u = r0_nm, species["rw_angstrom"], species["mass_u"]
    for k in range(LC_MAX_Z):
        d.ip_ev[k] = species["ip_ev"][k] if k < len(species["ip_ev"]) else 0.0
    d.intensity_wcm2 = intensity_wcm2
    d.envelope = ENVELOPES[envelope]
    d.phase = PHASES[phase]
    d.polarization = POLARIZATIONS[polarization]
    for k in range(LC_MAX_Z):
        d.lotz_q[k] = species.get("outer_q", [])[k] if k < len(species.get("outer_q", [])) else 0.0
    d.lotz_a = lotz_a
    d.fwhm_fs, d.n_cycles = fwhm_fs, n_cycles
    d.n_ion, d.capacity, d.weight, d.z_max = n_ion, capacity, weight, z_max
    d.electron_offset_nm, d.n_steps = electron_offset_nm, n_steps
    return d


class Simulation:
    """Clusters integrated by liblcmd on one GPU.

    The state lives in one torch uint8 tensor owned by this object; work runs on a torch
    stream of its own (default priority; graph capture needs a non-null stream), on which the
    state tensor is also allocated.
    """

    def __init__(self, config, clusters, device="cuda", stream=None):
        L = lib()
        self.config = config
        self.n_clusters = len(clusters)
        self._cl = (ClusterDesc * self.n_clusters)(*clusters)
        nbytes = L.lc_state_bytes(ctypes.byref(config), self._cl, self.n_clusters)
        if nbytes == 0:
            raise LcError(LC_E_INVALID, "invalid configuration (lc_state_bytes returned 0)")
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        with torch.cuda.stream(self.stream):
            self.state = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        code = L.lc_create(ctypes.byref(h), ctypes.byref(config), self._cl, self.n_clusters,
                           ctypes.c_void_p(self.state.data_ptr()), int(nbytes),
                           ctypes.c_void_p(self.stream.cuda_stream))
        _check(code)
        self.h = h
        self.capacity = [int(c.capacity) for c in clusters]

    def close(self):
        if getattr(self, "h", None):
            lib().lc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_from_host(self, cluster, x_nm, u, Z):
        x_nm = np.ascontiguousarray(x_nm, np.float64)
        u = np.ascontiguousarray(u, np.float64)
        Z = np.ascontiguousarray(Z, np.int8)
        n = x_nm.shape[0]
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().lc_init_from_host(self.h, cluster, n, x_nm.ctypes.data_as(dp), u.ctypes.data_as(dp),
                                       Z.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))), self.h)

    def init_generate(self, cluster=-1, z_init=1):
        """Seeded initial placement on the device (cluster -1: every cluster)."""
        _check(lib().lc_init_generate(self.h, int(cluster), int(z_init)), self.h)

    def start(self):
        _check(lib().lc_start(self.h), self.h)

    def step(self, n):
        _check(lib().lc_step(self.h, int(n)), self.h)

    def set_graph(self, steps_per_graph):
        _check(lib().lc_set_graph(self.h, int(steps_per_graph)), self.h)

    @property
    def step_index(self):
        return lib().lc_step_index(self.h)

    def diagnostics(self, cluster=0, max_records=None):
        mr = int(max_records or self.config.max_records)
        buf = np.zeros((max(mr, 1), LC_REC))
        n = ctypes.c_int32()
        _check(lib().lc_read_diagnostics(self.h, cluster, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), mr,
                                         ctypes.byref(n)), self.h)
        return buf[: n.value]

    def particles(self, cluster=0):
        cap = self.capacity[cluster]
        x = np.zeros((cap, 3))
        u = np.zeros((cap, 3))
        Z = np.zeros(cap, np.int8)
        wl = np.zeros(cap)
        wc = np.zeros(cap)
        n = ctypes.c_int64()
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().lc_read_particles(self.h, cluster, x.ctypes.data_as(dp), u.ctypes.data_as(dp),
                                       Z.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), wl.ctypes.data_as(dp),
                                       wc.ctypes.data_as(dp), cap, ctypes.byref(n)), self.h)
        k = n.value
        return {"x": x[:k], "u": u[:k], "Z": Z[:k], "wl": wl[:k], "wc": wc[:k], "n": k}

    def field(self, cluster=0):
        """Coulomb field (n x 3, field units) of a cluster's current positions, from a field pass
        with the current tiling (lc_read_field)."""
        cap = self.capacity[cluster]
        E = np.zeros((cap, 3))
        n = ctypes.c_int64()
        _check(lib().lc_read_field(self.h, cluster, E.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cap,
                                   ctypes.byref(n)), self.h)
        return E[:n.value]

    def iedf(self, cluster=0):
        """Detector counts (4 x LC_DET_SLOTS int64: every detected ion, then the x, y and z axes)
        and the LC_DET_BINS + 1 energy bin edges in eV (lc_read_iedf)."""
        counts = np.zeros((4, LC_DET_SLOTS), np.int64)
        edges = np.zeros(LC_DET_BINS + 1)
        _check(lib().lc_read_iedf(self.h, cluster, counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self.h)
        return counts, edges

    def time_particle_kernels(self, reps=20):
        """Average ms of the push kernel and of the ionization kernels (lc_time_particle_kernels)."""
        out = (ctypes.c_double * 2)()
        _check(lib().lc_time_particle_kernels(self.h, int(reps), out), self.h)
        return {"push_ms": out[0], "ionize_ms": out[1]}

    def counters(self, cluster=0):
        """(steps taken, live macroparticles, pair interactions evaluated, ionization events)."""
        out = (ctypes.c_double * 4)()
        _check(lib().lc_cluster_counters(self.h, cluster, out), self.h)
        return {"steps": int(out[0]), "n": int(out[1]), "pairs": out[2], "events": int(out[3])}

    def tuning(self):
        t = Tuning()
        _check(lib().lc_get_tuning(self.h, ctypes.byref(t)), self.h)
        return t.as_dict()

    def set_tuning(self, R=0, WJ=0, T=0, S=0, persistent=0, scalar=0, newton3=0):
        _check(lib().lc_set_tuning(self.h, ctypes.byref(make_tuning(R, WJ, T, S, persistent, scalar, newton3))),
               self.h)

    def autotune(self, cache_json=None):
        t = Tuning()
        _check(lib().lc_autotune(self.h, cache_json.encode() if cache_json else None, ctypes.byref(t)), self.h)
        return t.as_dict()

    def profile_steps(self, n):
        """Advance n steps with per-kernel-group HIP event timing: returns {group: (ms, launches)}."""
        ms = (ctypes.c_double * 4)()
        cnt = (ctypes.c_int64 * 4)()
        _check(lib().lc_profile_steps(self.h, int(n), ms, cnt), self.h)
        return {k: (ms[i], cnt[i]) for i, k in enumerate(["field", "push", "diag", "ionize"])}

    def save(self, path):
        _check(lib().lc_save_state(self.h, path.encode()), self.h)

    def load(self, path):
        _check(lib().lc_load_state(self.h, path.encode()), self.h)


LC_FIELD_STATIC_MAX_BYTES = 64 << 20


def field_static(xyzq, eps2, precision="fp64", want_phi=True, tuning=None):
    """As field(), through lc_field_static: no workspace is allocated (the library's device array
    serves as the workspace); only the outputs are allocated here.  Requests whose workspace would
    exceed LC_FIELD_STATIC_MAX_BYTES raise LcError."""
    L = lib()
    if xyzq.dtype != torch.float64 or not xyzq.is_cuda or xyzq.dim() != 2 or xyzq.shape[0] != 4:
        raise ValueError("xyzq must be a (4, n) float64 CUDA tensor")
    xyzq = xyzq.contiguous()
    n = xyzq.shape[1]
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    tp = ctypes.byref(tuning) if tuning is not None else None
    E = torch.empty((3, n), dtype=torch.float64, device=xyzq.device)
    phi = torch.empty(n, dtype=torch.float64, device=xyzq.device) if want_phi else None
    st = torch.cuda.current_stream(xyzq.device)
    code = L.lc_field_static(prec, n, ctypes.c_void_p(xyzq.data_ptr()), float(eps2), ctypes.c_void_p(E.data_ptr()),
                             ctypes.c_void_p(phi.data_ptr()) if want_phi else None, tp, ctypes.c_void_p(st.cuda_stream))
    _check(code)
    return E, phi


def field(xyzq, eps2, precision="fp64", want_phi=True, tuning=None):
    """Softened Coulomb field of n sources on themselves through lc_field.

    xyzq: CUDA float64 tensor of shape (4, n) (rows x, y, z, q).  Returns (E (3, n), phi (n) or None).
    """
    L = lib()
    if xyzq.dtype != torch.float64 or not xyzq.is_cuda or xyzq.dim() != 2 or xyzq.shape[0] != 4:
        raise ValueError("xyzq must be a (4, n) float64 CUDA tensor")
    xyzq = xyzq.contiguous()
    n = xyzq.shape[1]
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    t = tuning if tuning is not None else None
    tp = ctypes.byref(t) if t is not None else None
    wb = L.lc_field_workspace_bytes(prec, n, tp)
    if wb == 0:
        raise LcError(LC_E_INVALID, "invalid field request")
    work = torch.empty(int(wb), dtype=torch.uint8, device=xyzq.device)
    E = torch.empty((3, n), dtype=torch.float64, device=xyzq.device)
    phi = torch.empty(n, dtype=torch.float64, device=xyzq.device) if want_phi else None
    st = torch.cuda.current_stream(xyzq.device)
    code = L.lc_field(prec, n, ctypes.c_void_p(xyzq.data_ptr()), float(eps2), ctypes.c_void_p(E.data_ptr()),
                      ctypes.c_void_p(phi.data_ptr()) if want_phi else None, ctypes.c_void_p(work.data_ptr()),
                      int(wb), tp, ctypes.c_void_p(st.cuda_stream))
    _check(code)
    return E, phi


class Surrogate:
    """The 4-64-64-2 surrogate network on the GPU (lc_mlp_*).

    Its state (master weights, Adam moments, scaler, scratch) lives in one torch uint8 tensor;
    inputs and outputs are CUDA float32 tensors of shape (n, 4) and (n, 2).
    """

    def __init__(self, params, device="cuda", stream=None):
        L = lib()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        with torch.cuda.stream(self.stream):
            self.state = torch.empty(int(L.lc_mlp_state_bytes()), dtype=torch.uint8, device=self.device)
        self.set_params(params)

    def _st(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def _ptr(self, t):
        return ctypes.c_void_p(t.data_ptr())

    def set_params(self, params):
        p = np.ascontiguousarray(params, np.float32)
        if p.size != lib().lc_mlp_n_params():
            raise ValueError("wrong number of parameters")
        _check(lib().lc_mlp_set_params(self._ptr(self.state), p.ctypes.data_as(ctypes.c_void_p), self._st()))

    def params(self):
        p = np.zeros(lib().lc_mlp_n_params(), np.float32)
        sc = np.zeros(12, np.float32)
        _check(lib().lc_mlp_get_params(self._ptr(self.state), p.ctypes.data_as(ctypes.c_void_p),
                                       sc.ctypes.data_as(ctypes.c_void_p), self._st()))
        return p, {"x_mu": sc[0:4], "x_sd": sc[4:8], "y_mu": sc[8:10], "y_sd": sc[10:12]}

    @staticmethod
    def _check_xy(X, Y=None):
        if X.dtype != torch.float32 or not X.is_cuda or X.dim() != 2 or X.shape[1] != 4 or not X.is_contiguous():
            raise ValueError("X must be a contiguous (n, 4) float32 CUDA tensor")
        if Y is not None and (Y.dtype != torch.float32 or not Y.is_cuda or Y.shape != (X.shape[0], 2)
                              or not Y.is_contiguous()):
            raise ValueError("Y must be a contiguous (n, 2) float32 CUDA tensor")

    def _sync_inputs(self):
        # inputs were produced on torch's current stream; order the library's stream after it
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def fit_scaler(self, X, Y):
        self._check_xy(X, Y)
        self._sync_inputs()
        _check(lib().lc_mlp_fit_scaler(self._ptr(self.state), self._ptr(X), self._ptr(Y), X.shape[0], self._st()))

    def train(self, X, Y, rows, batch, steps, lr):
        self._check_xy(X, Y)
        if rows.dtype != torch.int32 or not rows.is_cuda or rows.numel() < steps * batch:
            raise ValueError("rows must be an int32 CUDA tensor of at least steps*batch entries")
        self._sync_inputs()
        with torch.cuda.stream(self.stream):
            loss = torch.empty(max(steps, 1), dtype=torch.float32, device=self.device)
        _check(lib().lc_mlp_train(self._ptr(self.state), self._ptr(X), self._ptr(Y), X.shape[0], self._ptr(rows),
                                  batch, steps, float(lr), self._ptr(loss), self._st()))
        _check(lib().lc_mlp_status(self._ptr(self.state), self._st()))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return loss[:steps]

    def grad(self, X, Y, rows, batch):
        self._check_xy(X, Y)
        self._sync_inputs()
        with torch.cuda.stream(self.stream):
            g = torch.empty(lib().lc_mlp_n_params(), dtype=torch.float32, device=self.device)
            loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _check(lib().lc_mlp_grad(self._ptr(self.state), self._ptr(X), self._ptr(Y), X.shape[0], self._ptr(rows),
                                 batch, self._ptr(g), self._ptr(loss), self._st()))
        self.stream.synchronize()
        return g, loss

    def infer(self, X):
        self._check_xy(X)
        self._sync_inputs()
        with torch.cuda.stream(self.stream):
            Y = torch.empty((X.shape[0], 2), dtype=torch.float32, device=self.device)
        _check(lib().lc_mlp_infer(self._ptr(self.state), self._ptr(X), self._ptr(Y), X.shape[0], self._st()))
        # hand the result to the caller's stream: its next use waits for the kernel
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return Y
