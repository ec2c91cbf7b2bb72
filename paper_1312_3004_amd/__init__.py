"""MI355X Replica-Exchange Wang-Landau (REWL) sampling.

Python binding of librewl.so, the HIP (gfx950) implementation of the parallel
Wang-Landau scheme of Vogel, Li, Wuest and Landau (J. Phys.: Conf. Ser.,
2014, Sec. 2): h overlapping energy windows, m walkers per window, replica
exchange between neighbouring windows (Eq. 1), window averaging at flat
histograms, and joining of the pieces (Fig. 2) -- here for the 2D q-state
Potts model of Eq. (2).

This module only marshals arguments.  Every step of the method runs in the
library's kernels; PyTorch provides the device workspace and the HIP stream.
The library must be built (``python -m paper_1312_3004_amd.build`` or
``__graft_entry__.build()``); importing the binding without it raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librewl.so")
# profiling build: the same library plus per-walker phase clocks of the
# attempt loop (include/rewl_phase_clocks.h)
CLOCKS_LIB_PATH = os.path.join(_HERE, "librewl_clocks.so")

OK, CONVERGED, EINVAL, ENOMEM, EDEVICE, ESTATE, EBUDGET = 0, 1, -1, -2, -3, -4, -5
POTTS2D, TRIMER3D = 0, 1


class RewlError(RuntimeError):
    pass


class Opts(ctypes.Structure):
    """Mirror of rewl_opts in include/rewl.h."""
    _fields_ = [("seed", ctypes.c_uint64), ("instance", ctypes.c_uint32),
                ("flat_num", ctypes.c_uint32), ("flat_den", ctypes.c_uint32),
                ("lnf_init", ctypes.c_double), ("lnf_final", ctypes.c_double),
                ("schedule", ctypes.c_int32), ("exchange", ctypes.c_int32),
                ("sync_attempts", ctypes.c_int64), ("precision", ctypes.c_int32),
                ("fixed_lnf", ctypes.c_int32), ("shadow", ctypes.c_int32),
                ("walkin_slack", ctypes.c_int32), ("obs_bins", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Instance(ctypes.Structure):
    """Mirror of rewl_instance in include/rewl.h."""
    _fields_ = [("model", ctypes.c_int32), ("L", ctypes.c_int32), ("q", ctypes.c_int32),
                ("windows", ctypes.c_int32), ("walkers", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("overlap", ctypes.c_double), ("opts", Opts)]


class Plan(ctypes.Structure):
    """Mirror of rewl_batch_plan in include/rewl.h."""
    _fields_ = [("walkers_per_cu", ctypes.c_int32), ("tag_policy", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("lds_bytes", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("resident", ctypes.c_int32), ("ms_per_step", ctypes.c_double), ("mixed", ctypes.c_int32),
                ("tag_bytes", ctypes.c_int32), ("slot_count", ctypes.c_int32 * 8), ("nclasses", ctypes.c_int32),
                ("class_lds", ctypes.c_int32 * 8)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["slot_count"] = list(self.slot_count)[: self.nclasses]
        d["class_lds"] = list(self.class_lds)[: self.nclasses]
        return d


_lib = None


def lib():
    """Load librewl.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1312_3004_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        L.rewl_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.rewl_default_opts.restype = None
        L.rewl_window_layout.argtypes = [i32, i32, dbl, P, P]
        L.rewl_workspace_bytes.argtypes = [i32, i32, i32, i32, dbl, i32, ctypes.POINTER(Opts)]
        L.rewl_workspace_bytes.restype = ctypes.c_size_t
        L.rewl_create.argtypes = [ctypes.POINTER(P), i32, i32, i32, i32, dbl, i32, ctypes.POINTER(Opts),
                                  P, P, ctypes.c_size_t, P]
        L.rewl_destroy.argtypes = [P]
        L.rewl_destroy.restype = None
        L.rewl_walkin.argtypes = [P, i64]
        L.rewl_run.argtypes = [P, i64]
        L.rewl_run_attempts.argtypes = [P, i64]
        L.rewl_exchange.argtypes = [P]
        L.rewl_get_progress.argtypes = [P, P, P, P]
        L.rewl_get_walker.argtypes = [P, i32, P, P, P, P, P, P]
        L.rewl_get_window.argtypes = [P, i32, P, P, P, P, P, P, P, P]
        L.rewl_get_state.argtypes = [P, i32, P, P, P, P, P]
        L.rewl_set_lng.argtypes = [P, i32, P]
        L.rewl_get_shadow.argtypes = [P, i32, P, P]
        L.rewl_get_replicas.argtypes = [P, P, P]
        L.rewl_get_replica_visits.argtypes = [P, i32, P]
        L.rewl_begin_production.argtypes = [P]
        L.rewl_get_obs.argtypes = [P, i32, P, P, P]
        L.rewl_obs_micro.argtypes = [P, P, P]
        L.rewl_obs_thermo.argtypes = [P, P, i32, P]
        flt = ctypes.c_float
        L.rewl_trimer_workspace_bytes.argtypes = [i32, flt, dbl, dbl, i32, i32, dbl, i32, ctypes.POINTER(Opts)]
        L.rewl_trimer_workspace_bytes.restype = ctypes.c_size_t
        L.rewl_create_trimer.argtypes = [ctypes.POINTER(P), i32, flt, dbl, dbl, i32, i32, dbl, i32,
                                         ctypes.POINTER(Opts), P, P, ctypes.c_size_t, P]
        L.rewl_window_layout_bins.argtypes = [i32, i32, dbl, P, P]
        L.rewl_lipid_workspace_bytes.argtypes = [i32, i32, flt, dbl, dbl, dbl, dbl, i32, i32, dbl, i32,
                                                 ctypes.POINTER(Opts)]
        L.rewl_lipid_workspace_bytes.restype = ctypes.c_size_t
        L.rewl_create_lipid.argtypes = [ctypes.POINTER(P), i32, i32, flt, dbl, dbl, dbl, dbl, i32, i32, dbl, i32,
                                        ctypes.POINTER(Opts), P, P, ctypes.c_size_t, P]
        L.rewl_get_particles.argtypes = [P, i32, P, P, P]
        L.rewl_lipid_structure.argtypes = [P, ctypes.c_size_t, P, ctypes.c_size_t, i32, i32, i32, flt, P, P]
        L.rewl_structure.argtypes = [P, P]
        L.rewl_structure_noalloc.argtypes = [P, P]
        L.rewl_lipid_obs_field.argtypes = [P, i32, dbl, dbl]
        L.rewl_get_energy.argtypes = [P, i32, ctypes.POINTER(dbl)]
        L.rewl_get_energy_fx.argtypes = [P, i32, ctypes.POINTER(ctypes.c_int64)]
        L.rewl_save.argtypes = [P, P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
        L.rewl_load.argtypes = [P, P, ctypes.c_size_t]
        L.rewl_get_lng.argtypes = [P, i32, P, i64, P, P]
        L.rewl_join.argtypes = [P, P, P]
        L.rewl_thermo.argtypes = [P, P, i32, P, P, P]
        L.rewl_set_timing.argtypes = [P, i32]
        L.rewl_get_timing.argtypes = [P, P, P, P, P]
        L.rewl_last_error.argtypes = []
        L.rewl_last_error.restype = ctypes.c_char_p
        IP, PP = ctypes.POINTER(Instance), ctypes.POINTER(Plan)
        L.rewl_batch_workspace_bytes.argtypes = [i32, IP]
        L.rewl_batch_workspace_bytes.restype = ctypes.c_size_t
        L.rewl_batch_create.argtypes = [ctypes.POINTER(P), i32, IP, P, P, ctypes.c_size_t, P]
        L.rewl_batch_destroy.argtypes = [P]
        L.rewl_batch_destroy.restype = None
        L.rewl_batch_instance.argtypes = [P, i32, ctypes.POINTER(P)]
        L.rewl_batch_walkin.argtypes = [P, i64]
        L.rewl_batch_set_plan.argtypes = [P, PP]
        L.rewl_batch_get_plan.argtypes = [P, PP]
        L.rewl_batch_tune.argtypes = [P, i32, PP, i32, ctypes.POINTER(i32)]
        L.rewl_batch_run.argtypes = [P, i64]
        L.rewl_batch_run_per_instance.argtypes = [P, i64]
        L.rewl_batch_progress.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i32)]
        L.rewl_batch_bootstrap_bytes.argtypes = [P, i32, i32]
        L.rewl_batch_bootstrap_bytes.restype = ctypes.c_size_t
        L.rewl_batch_bootstrap.argtypes = [P, i32, ctypes.c_uint64, P, i32, P, ctypes.c_size_t, P, P, P, P, P, P]
        L.rewl_batch_set_timing.argtypes = [P, i32]
        L.rewl_batch_get_timing.argtypes = [P, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
        if hasattr(L, "rewl_phase_clocks"):
            L.rewl_phase_clocks.argtypes = [P, ctypes.c_size_t, i32]
        _lib = L
    return _lib


def use_phase_clocks():
    """Load the profiling build librewl_clocks.so instead of librewl.so; call
    before anything else touches the library."""
    global LIB_PATH
    if _lib is not None and LIB_PATH != CLOCKS_LIB_PATH:
        raise RewlError("librewl.so is already loaded; use_phase_clocks() must come first")
    LIB_PATH = CLOCKS_LIB_PATH


PHASE_CLOCK_FIELDS = ("lane_cycles", "decide_cycles", "segments", "rounds", "exact_attempts", "blocks",
                      "round_cycles", "attempts", "setup_cycles", "commit_cycles", "exact_cycles", "tail_cycles")


def phase_clocks(rows, reset=False):
    """Per-walker phase counters of the profiling build, uint64 (rows, 12) in
    the order of PHASE_CLOCK_FIELDS; reset=True zeroes them afterwards."""
    L = lib()
    if not hasattr(L, "rewl_phase_clocks"):
        raise RewlError("phase clocks need the profiling build: call use_phase_clocks() first")
    out = np.zeros((rows, len(PHASE_CLOCK_FIELDS)), dtype=np.uint64)
    _check(L.rewl_phase_clocks(_ptr(out), rows, int(reset)))
    return out


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(status):
    if status < 0:
        raise RewlError(f"librewl error {status}: {lib().rewl_last_error().decode()}")
    return status


def default_opts():
    o = Opts()
    lib().rewl_default_opts(ctypes.byref(o))
    return o


def window_layout(L, windows, overlap):
    """(W, starts) of the energy-range splitting (Sec. 2, Fig. 1)."""
    W = ctypes.c_int32(0)
    starts = np.zeros(windows, dtype=np.int32)
    _check(lib().rewl_window_layout(L, windows, overlap, ctypes.byref(W), _ptr(starts)))
    return W.value, starts


def make_opts(seed=1, instance=0, flat=(4, 5), lnf_init=1.0, lnf_final=1e-6, schedule=0,
              sync_attempts=1000, exchange=1, precision=0, fixed_lnf=0, shadow=0, walkin_slack=16, obs_bins=0):
    o = default_opts()
    o.seed, o.instance = seed, instance
    o.flat_num, o.flat_den = flat
    o.lnf_init, o.lnf_final = lnf_init, lnf_final
    o.schedule, o.sync_attempts, o.exchange = schedule, sync_attempts, exchange
    o.precision, o.fixed_lnf, o.shadow = precision, fixed_lnf, shadow
    o.walkin_slack = walkin_slack
    o.obs_bins = obs_bins
    return o


def workspace_bytes(L, q, windows, overlap, walkers, opts):
    return lib().rewl_workspace_bytes(POTTS2D, L, q, windows, overlap, walkers, ctypes.byref(opts))


class Rewl:
    """One REWL run of the 2D q-state Potts model on the GPU.

    ``init_spins``: int8 array [windows*walkers, L*L] of starting lattices.
    Keyword options mirror rewl_opts.  ``device``: torch device of the
    workspace (default cuda:0); ``stream``: torch.cuda.Stream to enqueue on
    (default: the device's current stream).
    """

    def __init__(self, L, q, windows, overlap, walkers, init_spins, device=None, stream=None, **opts):
        import torch

        self._describe(L, q, windows, overlap, walkers, make_opts(**opts))
        spins = np.ascontiguousarray(init_spins, dtype=np.int8).reshape(-1)
        if spins.size != self.nw * self.N:
            raise ValueError("init_spins must hold one L*L lattice per walker")
        nbytes = workspace_bytes(L, q, windows, overlap, walkers, self.opts)
        if nbytes == 0:
            _check(lib().rewl_create(ctypes.byref(ctypes.c_void_p()), POTTS2D, L, q, windows, overlap,
                                     walkers, ctypes.byref(self.opts), None, None, 0, None))
        self.device = torch.device(device if device is not None else "cuda:0")
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().rewl_create(ctypes.byref(h), POTTS2D, L, q, windows, overlap, walkers,
                                     ctypes.byref(self.opts), _ptr(spins),
                                     ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                     ctypes.c_void_p(self._stream.cuda_stream)))
        self._h = h

    def _describe(self, L, q, windows, overlap, walkers, opts):
        self.L, self.q, self.h, self.m = L, q, windows, walkers
        self.N = L * L
        self.nw = windows * walkers
        self.opts = opts
        self.precision, self.obs_bins = self.opts.precision, self.opts.obs_bins
        self.W, self.starts = window_layout(L, windows, overlap)
        self.B = 2 * self.N + 1
        self.e_lo = -2 * self.N

    @classmethod
    def trimer(cls, nmol, box, e_min, bin_w, bins, windows, overlap, walkers, init_coords, device=None,
               stream=None, **opts):
        """A run of the trimer model; init_coords: float32 [windows*walkers, 3 nmol, 3]."""
        import torch

        self = cls.__new__(cls)
        o = make_opts(**opts)
        self.h, self.m, self.nw = windows, walkers, windows * walkers
        self.opts, self.precision, self.obs_bins = o, o.precision, o.obs_bins
        self.nmol, self.box, self.e_min, self.bin_w = nmol, box, e_min, bin_w
        self.L = self.q = 0
        self.N = 9 * nmol * 4
        self.B, self.e_lo = bins, 0
        W = ctypes.c_int32(0)
        self.starts = np.zeros(windows, dtype=np.int32)
        _check(lib().rewl_window_layout_bins(bins, windows, overlap, ctypes.byref(W), _ptr(self.starts)))
        self.W = W.value
        x = np.ascontiguousarray(init_coords, dtype=np.float32).reshape(-1)
        if x.size != self.nw * 9 * nmol:
            raise ValueError("init_coords must hold 3 nmol beads x 3 coordinates per walker")
        args = (nmol, box, e_min, bin_w, bins, windows, overlap, walkers, ctypes.byref(o))
        nbytes = lib().rewl_trimer_workspace_bytes(*args)
        if nbytes == 0:
            _check(lib().rewl_create_trimer(ctypes.byref(ctypes.c_void_p()), *args, _ptr(x), None, 0, None))
        self.device = torch.device(device if device is not None else "cuda:0")
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().rewl_create_trimer(ctypes.byref(h), *args, _ptr(x),
                                            ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                            ctypes.c_void_p(self._stream.cuda_stream)))
        self._h = h
        return self

    @classmethod
    def lipid(cls, nlip, nsol, box, e_min, bin_w, bins, windows, overlap, walkers, init_coords, eps_ww=1.0,
              rep_prob=None, device=None, stream=None, **opts):
        """A run of the lipid model with explicit solvent; init_coords float32 [windows*walkers, np, 3].

        rep_prob: reptation probability per update (default 3 nlip / (10 np))."""
        import torch

        self = cls.__new__(cls)
        o = make_opts(**opts)
        self.h, self.m, self.nw = windows, walkers, windows * walkers
        self.opts, self.precision, self.obs_bins = o, o.precision, o.obs_bins
        self.nlip, self.np, self.box, self.e_min, self.bin_w = nlip, 3 * nlip + nsol, box, e_min, bin_w
        self.L = self.q = 0
        # bytes of a walker's state row: coordinates, types (padded to 4), lipid rows, position table
        self.N = 12 * self.np + (self.np + 3) // 4 * 4 + 12 * nlip + 4 * self.np
        self.B, self.e_lo = bins, 0
        W = ctypes.c_int32(0)
        self.starts = np.zeros(windows, dtype=np.int32)
        _check(lib().rewl_window_layout_bins(bins, windows, overlap, ctypes.byref(W), _ptr(self.starts)))
        self.W = W.value
        x = np.ascontiguousarray(init_coords, dtype=np.float32).reshape(-1)
        if x.size != self.nw * 3 * self.np:
            raise ValueError("init_coords must hold np particles x 3 coordinates per walker")
        rp = -1.0 if rep_prob is None else float(rep_prob)
        args = (nlip, nsol, box, eps_ww, rp, e_min, bin_w, bins, windows, overlap, walkers, ctypes.byref(o))
        nbytes = lib().rewl_lipid_workspace_bytes(*args)
        if nbytes == 0:
            _check(lib().rewl_create_lipid(ctypes.byref(ctypes.c_void_p()), *args, _ptr(x), None, 0, None))
        self.device = torch.device(device if device is not None else "cuda:0")
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().rewl_create_lipid(ctypes.byref(h), *args, _ptr(x),
                                           ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                           ctypes.c_void_p(self._stream.cuda_stream)))
        self._h = h
        return self

    def lipid_state(self, w):
        """(coords float32 [np, 3], types int8 [np] (0 P, 1 H, 2 W), lipids int32 [nlip, 3])."""
        x = np.zeros((self.np, 3), dtype=np.float32)
        t = np.zeros(self.np, dtype=np.int8)
        lp = np.zeros((self.nlip, 3), dtype=np.int32)
        _check(lib().rewl_get_particles(self._h, w, _ptr(x), _ptr(t), _ptr(lp)))
        return x, t, lp

    def structure(self):
        """Structural observables (Eqs. 6-8) of every walker's configuration: float64 [walkers, 8]
        = (S_mol, axis, clusters, largest, Q_xx, Q_yy, Q_zz, prolateness)."""
        out = np.zeros((self.nw, 8), dtype=np.float64)
        _check(lib().rewl_structure(self._h, _ptr(out)))
        return out

    def structure_noalloc(self):
        """structure() through the entry point that allocates no device memory (static record buffer)."""
        out = np.zeros((self.nw, 8), dtype=np.float64)
        _check(lib().rewl_structure_noalloc(self._h, _ptr(out)))
        return out

    def lipid_obs_field(self, field, lo=0.0, hi=0.0):
        """Record field binned as O in H(E, O): 3 (largest cluster, the default), or 0, 4-7
        (S_mol, Q_xx, Q_yy, Q_zz, prolateness) in obs_bins bins over [lo, hi)."""
        _check(lib().rewl_lipid_obs_field(self._h, int(field), float(lo), float(hi)))

    def save(self):
        """Checkpoint of the whole run (bytes)."""
        n = ctypes.c_size_t(0)
        _check(lib().rewl_save(self._h, None, 0, ctypes.byref(n)))
        buf = np.zeros(n.value, dtype=np.uint8)
        _check(lib().rewl_save(self._h, _ptr(buf), n.value, ctypes.byref(n)))
        return buf.tobytes()

    def load(self, blob):
        """Restore a checkpoint written by save() of a run with the same sizes and options."""
        buf = np.frombuffer(blob, dtype=np.uint8)
        _check(lib().rewl_load(self._h, _ptr(buf), buf.size))

    def energy(self, w):
        """Energy of walker w (the trimer model's continuous energy)."""
        e = ctypes.c_double(0)
        _check(lib().rewl_get_energy(self._h, w, ctypes.byref(e)))
        return e.value

    def energy_fx(self, w):
        """Energy of walker w in units of 2^-32 (continuous models; the Potts energy for Potts runs)."""
        e = ctypes.c_int64(0)
        _check(lib().rewl_get_energy_fx(self._h, w, ctypes.byref(e)))
        return e.value

    @classmethod
    def _view(cls, handle, L, q, windows, overlap, walkers, opts, owner):
        """A Rewl over an instance handle owned by a Batch."""
        self = cls.__new__(cls)
        self._describe(L, q, windows, overlap, walkers, opts)
        self._h = handle
        self._owner = owner
        return self

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and getattr(self, "_owner", None) is None and _lib is not None:
            _lib.rewl_destroy(h)
            self._h = None

    @property
    def stream(self):
        return self._stream

    def walkin(self, budget=1 << 40):
        return _check(lib().rewl_walkin(self._h, int(budget)))

    def run(self, attempts):
        """Run `attempts` more attempts per walker; returns OK or CONVERGED."""
        return _check(lib().rewl_run_attempts(self._h, int(attempts)))

    def run_sweeps(self, sweeps):
        return _check(lib().rewl_run(self._h, int(sweeps)))

    def exchange(self):
        return _check(lib().rewl_exchange(self._h))

    def progress(self):
        s, r, c = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int32(0)
        _check(lib().rewl_get_progress(self._h, ctypes.byref(s), ctypes.byref(r), ctypes.byref(c)))
        return s.value, r.value, bool(c.value)

    @property
    def step(self):
        return self.progress()[0]

    @property
    def round(self):
        return self.progress()[1]

    def walker(self, w):
        spins = np.zeros(self.N, dtype=np.int8)
        E = ctypes.c_int32(0)
        H = np.zeros(self.W, dtype=np.uint32)
        lng = np.zeros(self.W)
        rep = ctypes.c_uint32(0)
        wa = ctypes.c_int64(0)
        _check(lib().rewl_get_walker(self._h, w, _ptr(spins), ctypes.byref(E), _ptr(H), _ptr(lng),
                                     ctypes.byref(rep), ctypes.byref(wa)))
        return dict(spins=spins, E=E.value, H=H, lng=lng, replica=rep.value, walkin_attempts=wa.value)

    def state(self, w):
        """Walker w's spins, E, H, ln g and its window's current ln f in one call."""
        spins = np.zeros(self.N, dtype=np.int8)
        E = ctypes.c_int32(0)
        H = np.zeros(self.W, dtype=np.uint32)
        lng = np.zeros(self.W)
        lnf = ctypes.c_double(0)
        _check(lib().rewl_get_state(self._h, w, _ptr(spins), ctypes.byref(E), _ptr(H), _ptr(lng),
                                    ctypes.byref(lnf)))
        return dict(spins=spins, E=E.value, H=H, lng=lng, lnf=lnf.value)

    def window(self, k):
        lnf, lnf_last = ctypes.c_double(0), ctypes.c_double(0)
        regime, fin = ctypes.c_int32(0), ctypes.c_int32(0)
        it = ctypes.c_int64(0)
        vis = np.zeros(self.W, dtype=np.uint8)
        xa, xc = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(lib().rewl_get_window(self._h, k, ctypes.byref(lnf), ctypes.byref(lnf_last),
                                     ctypes.byref(regime), ctypes.byref(fin), ctypes.byref(it), _ptr(vis),
                                     ctypes.byref(xa), ctypes.byref(xc)))
        return dict(lnf=lnf.value, lnf_last=lnf_last.value, regime=regime.value, finished=fin.value,
                    iterations=it.value, visited=vis, x_att=xa.value, x_acc=xc.value)

    def replicas(self):
        """(window_of, trips), uint32 [h*m] by replica id: current window and completed round trips."""
        win = np.zeros(self.nw, dtype=np.uint32)
        trips = np.zeros(self.nw, dtype=np.uint32)
        _check(lib().rewl_get_replicas(self._h, _ptr(win), _ptr(trips)))
        return win, trips

    def begin_production(self):
        """Freeze the current ln g as weights (ln f = 0 everywhere), no termination, restart H."""
        _check(lib().rewl_begin_production(self._h))

    def obs(self, w):
        """Walker w's H(E, O) [W, obs_bins], sum of O [W] and samples [W]."""
        hist = np.zeros((self.W, self.obs_bins), dtype=np.uint32)
        s = np.zeros(self.W, dtype=np.uint64)
        c = np.zeros(self.W, dtype=np.uint32)
        _check(lib().rewl_get_obs(self._h, w, _ptr(hist), _ptr(s), _ptr(c)))
        return hist, s, c

    def obs_micro(self):
        """(mean O [B], samples [B]) pooled over the walkers of every window holding the bin."""
        mean = np.zeros(self.B)
        cnt = np.zeros(self.B, dtype=np.uint64)
        _check(lib().rewl_obs_micro(self._h, _ptr(mean), _ptr(cnt)))
        return mean, cnt

    def obs_thermo(self, T):
        """Canonical average of O on the temperature grid T (needs a current join)."""
        T = np.ascontiguousarray(T, dtype=np.float64)
        out = np.zeros_like(T)
        _check(lib().rewl_obs_thermo(self._h, _ptr(T), len(T), _ptr(out)))
        return out

    def replica_visits(self, w):
        """uint32 [h*m]: lookups that found each replica id in walker slot w."""
        out = np.zeros(self.nw, dtype=np.uint32)
        _check(lib().rewl_get_replica_visits(self._h, w, _ptr(out)))
        return out

    def shadow(self, w):
        """(hi, lo): double-double exact reference of walker w's ln g (opts shadow=1)."""
        hi, lo = np.zeros(self.W), np.zeros(self.W)
        _check(lib().rewl_get_shadow(self._h, w, _ptr(hi), _ptr(lo)))
        return hi, lo

    def set_lng(self, w, lng):
        a = np.ascontiguousarray(lng, dtype=np.float64)
        if a.size != self.W:
            raise ValueError("ln g must have W entries")
        _check(lib().rewl_set_lng(self._h, w, _ptr(a)))

    def get_lng(self, k):
        """ln g of window k (walker 0), -inf where unvisited; k = -1: joined."""
        n = self.B if k == -1 else self.W
        out = np.zeros(n)
        nn, ef = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib().rewl_get_lng(self._h, k, _ptr(out), n, ctypes.byref(nn), ctypes.byref(ef)))
        return out[: nn.value], ef.value

    def join(self):
        """(status, joined ln g over 2N+1 energies, joining energies)."""
        out = np.zeros(self.B)
        cuts = np.zeros(max(self.h - 1, 1), dtype=np.int32)
        st = lib().rewl_join(self._h, _ptr(out), _ptr(cuts))
        if st < 0 and st != ESTATE:
            _check(st)
        return st, out, cuts[: self.h - 1]

    def set_timing(self, enable=True):
        _check(lib().rewl_set_timing(self._h, 1 if enable else 0))

    def timing(self):
        """(attempt-kernel ms, launches, sync-point ms, sync points) since set_timing."""
        a, b = ctypes.c_double(0), ctypes.c_int64(0)
        c, d = ctypes.c_double(0), ctypes.c_int64(0)
        _check(lib().rewl_get_timing(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                     ctypes.byref(d)))
        return a.value, b.value, c.value, d.value

    def thermo(self, T):
        T = np.ascontiguousarray(T, dtype=np.float64)
        lnZ, U, C = np.zeros_like(T), np.zeros_like(T), np.zeros_like(T)
        _check(lib().rewl_thermo(self._h, _ptr(T), len(T), _ptr(lnZ), _ptr(U), _ptr(C)))
        return lnZ, U, C


class Batch:
    """Many independent REWL runs advanced together (the batched form).

    ``instances``: list of dicts with keys L, q, windows, overlap, walkers and
    any rewl_opts option (seed, instance, flat, lnf_init, ...).
    ``init_spins``: list of int8 arrays, one [windows*walkers, L*L] per instance.
    """

    def __init__(self, instances, init_spins, device=None, stream=None):
        import torch

        n = len(instances)
        arr = (Instance * n)()
        self._desc = []
        for i, d in enumerate(instances):
            d = dict(d)
            geo = {k: d.pop(k) for k in ("L", "q", "windows", "overlap", "walkers")}
            o = make_opts(**d)
            arr[i].model = POTTS2D
            arr[i].L, arr[i].q, arr[i].windows, arr[i].walkers = geo["L"], geo["q"], geo["windows"], geo["walkers"]
            arr[i].overlap = geo["overlap"]
            arr[i].opts = o
            self._desc.append((geo, o))
        self._arr = arr
        self.n = n
        spins = np.concatenate([np.ascontiguousarray(s, dtype=np.int8).reshape(-1) for s in init_spins])
        nbytes = lib().rewl_batch_workspace_bytes(n, arr)
        self.device = torch.device(device if device is not None else "cuda:0")
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if nbytes == 0:
            _check(lib().rewl_batch_create(ctypes.byref(ctypes.c_void_p()), n, arr, _ptr(spins), None, 0, None))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().rewl_batch_create(ctypes.byref(h), n, arr, _ptr(spins),
                                           ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                           ctypes.c_void_p(self._stream.cuda_stream)))
        self._h = h
        self._views = [None] * n

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.rewl_batch_destroy(h)
            self._h = None

    def bootstrap(self, nboot, seed, T=()):
        """Bootstrap over the instances (independent converged runs of one system).

        Returns a dict: lng_mean, lng_std [B]; U_mean, U_std, C_mean, C_std [len(T)]."""
        import torch

        T = np.ascontiguousarray(T, dtype=np.float64)
        nT = len(T)
        nbytes = lib().rewl_batch_bootstrap_bytes(self._h, int(nboot), nT)
        if nbytes == 0:
            raise RewlError("invalid bootstrap arguments")
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        B = 2 * self._desc[0][0]["L"] ** 2 + 1
        out = {k: np.zeros(B) for k in ("lng_mean", "lng_std")}
        out.update({k: np.zeros(nT) for k in ("U_mean", "U_std", "C_mean", "C_std")})
        with torch.cuda.device(self.device):
            _check(lib().rewl_batch_bootstrap(self._h, int(nboot), int(seed), _ptr(T), nT,
                                              ctypes.c_void_p(scratch.data_ptr()), nbytes, _ptr(out["lng_mean"]),
                                              _ptr(out["lng_std"]), _ptr(out["U_mean"]), _ptr(out["U_std"]),
                                              _ptr(out["C_mean"]), _ptr(out["C_std"])))
        self._stream.synchronize()
        return out

    def instance(self, i):
        """Rewl view of instance i (walker/window/join/thermo queries)."""
        if self._views[i] is None:
            ih = ctypes.c_void_p()
            _check(lib().rewl_batch_instance(self._h, i, ctypes.byref(ih)))
            geo, o = self._desc[i]
            self._views[i] = Rewl._view(ih, geo["L"], geo["q"], geo["windows"], geo["overlap"], geo["walkers"],
                                        o, self)
        return self._views[i]

    def walkin(self, budget=1 << 40):
        return _check(lib().rewl_batch_walkin(self._h, int(budget)))

    def run(self, steps):
        """`steps` batched steps (one sync interval of every instance each)."""
        return _check(lib().rewl_batch_run(self._h, int(steps)))

    def run_per_instance(self, steps):
        return _check(lib().rewl_batch_run_per_instance(self._h, int(steps)))

    def plan(self):
        p = Plan()
        _check(lib().rewl_batch_get_plan(self._h, ctypes.byref(p)))
        return p.as_dict()

    def set_plan(self, walkers_per_cu=0, tag_policy=0, use_graph=1, slot_count=None, tag_bytes=4096):
        """Uniform plan, or with slot_count (slots per CU per class, largest class
        first) the mixed-slot plan."""
        p = Plan()
        p.walkers_per_cu, p.tag_policy, p.use_graph = walkers_per_cu, tag_policy, use_graph
        if slot_count is not None:
            p.mixed, p.tag_bytes = 1, tag_bytes
            for i, c in enumerate(slot_count):
                p.slot_count[i] = c
        _check(lib().rewl_batch_set_plan(self._h, ctypes.byref(p)))
        return p.as_dict()

    def tune(self, steps_per_plan=1, cap=256):
        """Autotune the launch plan; returns (chosen plan, list of trials)."""
        tried = (Plan * cap)()
        nt = ctypes.c_int32(0)
        _check(lib().rewl_batch_tune(self._h, int(steps_per_plan), tried, cap, ctypes.byref(nt)))
        return self.plan(), [tried[i].as_dict() for i in range(nt.value)]

    def progress(self):
        s, c = ctypes.c_int64(0), ctypes.c_int32(0)
        _check(lib().rewl_batch_progress(self._h, ctypes.byref(s), ctypes.byref(c)))
        return s.value, c.value

    def set_timing(self, enable=True):
        _check(lib().rewl_batch_set_timing(self._h, 1 if enable else 0))

    def timing(self):
        """(milliseconds, batched steps) since set_timing."""
        ms, n = ctypes.c_double(0), ctypes.c_int64(0)
        _check(lib().rewl_batch_get_timing(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


def lipid_structure(coords, lipids, box, out=None, stream=None):
    """Structural observables (Sec. 3.2, Eqs. 6-8) of lipid configurations on the GPU.

    coords: CUDA float32 [nconf, np, 3]; lipids: CUDA int32 [nconf, nlip, 3]
    (particle indices, head first), both contiguous.  Returns CUDA float64
    [nconf, 8] = (S_mol, axis, clusters, largest, Q_xx, Q_yy, Q_zz,
    prolateness), queued on ``stream`` (default: the current stream)."""
    import torch

    if coords.dim() != 3 or coords.shape[2] != 3 or lipids.dim() != 3 or lipids.shape[2] != 3:
        raise ValueError("coords must be [nconf, np, 3] and lipids [nconf, nlip, 3]")
    if coords.dtype != torch.float32 or lipids.dtype != torch.int32:
        raise TypeError("coords must be float32 and lipids int32")
    if not (coords.is_cuda and lipids.is_cuda) or not (coords.is_contiguous() and lipids.is_contiguous()):
        raise ValueError("coords and lipids must be contiguous CUDA tensors")
    nconf, np_, nlip = coords.shape[0], coords.shape[1], lipids.shape[1]
    if lipids.shape[0] != nconf:
        raise ValueError("coords and lipids hold different numbers of configurations")
    if out is None:
        out = torch.empty((nconf, 8), dtype=torch.float64, device=coords.device)
    elif out.shape != (nconf, 8) or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 [nconf, 8] tensor")
    s = stream if stream is not None else torch.cuda.current_stream(coords.device)
    _check(lib().rewl_lipid_structure(ctypes.c_void_p(coords.data_ptr()), 12 * np_,
                                      ctypes.c_void_p(lipids.data_ptr()), 12 * nlip, nconf, np_, nlip,
                                      float(box), ctypes.c_void_p(out.data_ptr()),
                                      ctypes.c_void_p(s.cuda_stream)))
    return out
