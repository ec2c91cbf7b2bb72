"""CPU oracle for Replica-Exchange Wang-Landau sampling (test infrastructure).

Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product library never loads it: it exists to prove
the GPU path right.  The arithmetic lives in rewl_oracle.c (plain C, binary64,
no FMA); this module only loads that library and marshals arguments, plus the
brute-force density of states in bruteforce.py and the lipid model's
structural observables (numpy) in structure.py.
"""
import ctypes
import os

import numpy as np

from . import build as _build

OK, CONVERGED, EINVAL, ENOMEM, ESTATE, EBUDGET = 0, 1, -1, -2, -4, -5

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64, u32, u64, dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        L.orc_create.restype = P
        L.orc_create.argtypes = [i32, i32, i32, dbl, i32, u64, u32, u32, u32, dbl, dbl, i32, i64,
                                 i32, i32, i32, i32, i32, i32, P]
        L.orc_begin_production.argtypes = [P]
        L.orc_begin_production.restype = i32
        L.orc_get_obs.argtypes = [P, i32, P, P, P]
        L.orc_get_obs.restype = i32
        L.orc_obs_micro.argtypes = [P, P, P]
        L.orc_obs_micro.restype = i32
        L.orc_obs_thermo.argtypes = [P, P, i32, dbl, dbl, P, i32, P]
        L.orc_obs_thermo.restype = None
        L.orc_bootstrap.argtypes = [i32, i32, i32, P, i32, i32, P, P, dbl, i32, u64, P, i32, dbl, dbl,
                                    P, P, P, P, P, P]
        L.orc_bootstrap.restype = i32
        L.orc_create_lipid.restype = P
        L.orc_create_lipid.argtypes = [i32, i32, ctypes.c_float, dbl, u32, dbl, dbl, i32, i32, dbl, i32, u64, u32,
                                       u32, u32, dbl, dbl, i32, i64, i32, i32, i32, P]
        L.orc_lipid_energy_fx.argtypes = [P, i32, ctypes.POINTER(i64)]
        L.orc_lipid_energy_fx.restype = i32
        L.orc_log_poly.argtypes = [dbl]
        L.orc_log_poly.restype = dbl
        L.orc_lipid_pair.argtypes = [P, i32, i32, i32, dbl]
        L.orc_lipid_pair.restype = dbl
        L.orc_lipid_state.argtypes = [P, i32, P, P, P]
        L.orc_lipid_state.restype = None
        L.orc_lipid_delta_move_fx.argtypes = [P, i32, i32, P, ctypes.POINTER(i64)]
        L.orc_lipid_delta_move_fx.restype = i32
        L.orc_lipid_reptate.argtypes = [P, i32, i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                        ctypes.POINTER(i64)]
        L.orc_lipid_reptate.restype = i32
        L.orc_get_shadow.argtypes = [P, i32, P, P]
        L.orc_get_replicas.argtypes = [P, P, P]
        L.orc_get_replicas.restype = None
        L.orc_get_replica_visits.argtypes = [P, i32, P]
        L.orc_create_trimer.restype = P
        L.orc_create_trimer.argtypes = [i32, ctypes.c_float, dbl, dbl, i32, i32, dbl, i32, u64, u32, u32,
                                        u32, dbl, dbl, i32, i64, i32, i32, i32, i32, i32, P]
        L.orc_get_energy.argtypes = [P, i32]
        L.orc_get_energy.restype = dbl
        L.orc_get_energy_fx.argtypes = [P, i32]
        L.orc_get_energy_fx.restype = i64
        L.orc_trimer_energy_fx.argtypes = [P, i32, ctypes.POINTER(i64)]
        L.orc_trimer_energy_fx.restype = i32
        L.orc_trimer_delta_fx.argtypes = [P, i32, i32, P, ctypes.POINTER(i64)]
        L.orc_trimer_delta_fx.restype = i32
        L.orc_get_shadow.restype = None
        for name, args in (("orc_dd_add", [P, P, dbl, dbl]), ("orc_dd_div_int", [P, P, i32]),
                           ("orc_dd_mul_count", [u32, dbl, P, P])):
            getattr(L, name).argtypes = args
            getattr(L, name).restype = None
        L.orc_destroy.argtypes = [P]
        L.orc_set_threads.argtypes = [P, i32]
        L.orc_walkin.argtypes = [P, i64]
        L.orc_walkin.restype = i32
        L.orc_run.argtypes = [P, i64, i64]
        L.orc_run.restype = i32
        L.orc_exchange.argtypes = [P]
        L.orc_exchange.restype = i32
        L.orc_info.argtypes = [P, P]
        L.orc_starts.argtypes = [P, P]
        L.orc_get_walker.argtypes = [P, i32, P, P, P, P, P, P, P, P]
        L.orc_get_window.argtypes = [P, i32, P, P, P, P, P, P, P, P]
        L.orc_set_lng.argtypes = [P, i32, P]
        L.orc_plant_walker.argtypes = [P, i32, P, P]
        L.orc_set_step.argtypes = [P, i64]
        L.orc_set_window.argtypes = [P, i32, dbl, i32]
        L.orc_sync_window.argtypes = [P, i32]
        L.orc_join.argtypes = [P, P, P]
        L.orc_join.restype = i32
        L.orc_join_pieces.argtypes = [i32, i32, P, i32, i32, P, P, dbl, P, P]
        L.orc_join_pieces.restype = i32
        L.orc_thermo.argtypes = [P, i32, dbl, dbl, P, i32, P, P, P]
        L.orc_philox.argtypes = [P, P, P]
        L.orc_exp_poly.argtypes = [dbl]
        L.orc_exp_poly.restype = dbl
        L.orc_exp_poly32.argtypes = [ctypes.c_float]
        L.orc_exp_poly32.restype = ctypes.c_float
        L.orc_window_layout.argtypes = [i32, i32, dbl, i32, P, P]
        L.orc_window_layout.restype = i32
        L.orc_potts_energy.argtypes = [P, i32]
        L.orc_potts_energy.restype = i32
        L.orc_constants.argtypes = [P]
        L.orc_constants32.argtypes = [P]
        L.orc_twosum_accumulate.argtypes = [P, P, ctypes.c_float, i64]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


FX_ONE = 2.0**32   # continuous-model energies are integers in units of 2^-32


def fx_to_float(e):
    """Nearest binary64 of an energy given in units of 2^-32."""
    return float(np.float64(e) / FX_ONE)


def philox(ctr, key):
    """Philox4x32-10 block: ctr = 4 uint32 words, key = 2 uint32 words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def exp_poly(x):
    return lib().orc_exp_poly(float(x))


def exp_poly32(x):
    return lib().orc_exp_poly32(float(np.float32(x)))


def constants():
    c = np.zeros(3)
    lib().orc_constants(_ptr(c))
    return c


def constants32():
    c = np.zeros(3, dtype=np.float32)
    lib().orc_constants32(_ptr(c))
    return c


def twosum_accumulate(hi, lo, x, n):
    a = np.array([hi], dtype=np.float32)
    b = np.array([lo], dtype=np.float32)
    lib().orc_twosum_accumulate(_ptr(a), _ptr(b), float(np.float32(x)), int(n))
    return float(a[0]), float(b[0])


def dd_add(a, b):
    """Double-double sum of (hi, lo) pairs a and b."""
    hi, lo = ctypes.c_double(a[0]), ctypes.c_double(a[1])
    lib().orc_dd_add(ctypes.byref(hi), ctypes.byref(lo), b[0], b[1])
    return hi.value, lo.value


def dd_div_int(a, m):
    hi, lo = ctypes.c_double(a[0]), ctypes.c_double(a[1])
    lib().orc_dd_div_int(ctypes.byref(hi), ctypes.byref(lo), m)
    return hi.value, lo.value


def dd_mul_count(n, x):
    hi, lo = ctypes.c_double(0), ctypes.c_double(0)
    lib().orc_dd_mul_count(n, x, ctypes.byref(hi), ctypes.byref(lo))
    return hi.value, lo.value


def window_layout(B, h, overlap, e_lo):
    W = ctypes.c_int(0)
    starts = np.zeros(h, dtype=np.int32)
    st = lib().orc_window_layout(B, h, overlap, e_lo, ctypes.byref(W), _ptr(starts))
    if st != OK:
        raise ValueError("invalid window layout")
    return W.value, starts


def potts_energy(spins, L):
    s = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1)
    return lib().orc_potts_energy(_ptr(s), L)


def thermo(lng, e_first, T, de=1.0):
    """ln Z, U, C_v on the grid T; bin b stands for energy e_first + b de."""
    g = np.ascontiguousarray(lng, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    lnZ, U, C = np.zeros_like(T), np.zeros_like(T), np.zeros_like(T)
    lib().orc_thermo(_ptr(g), len(g), float(e_first), float(de), _ptr(T), len(T), _ptr(lnZ), _ptr(U),
                     _ptr(C))
    return lnZ, U, C


def bootstrap(pieces, visited, starts, e_lo, B, log_total, nboot, seed, T, e_first=None, de=1.0):
    """Bootstrap over R runs: pieces float64 [R, h, W], visited uint8 [R, h, W].

    Returns (status, dict of lng_mean, lng_std [B], U_mean, U_std, C_mean, C_std [nT])."""
    p = np.ascontiguousarray(pieces, dtype=np.float64)
    v = np.ascontiguousarray(visited, dtype=np.uint8)
    R, h, W = p.shape
    starts = np.ascontiguousarray(starts, dtype=np.int32)
    T = np.ascontiguousarray(T, dtype=np.float64)
    out = {k: np.zeros(B) for k in ("lng_mean", "lng_std")}
    out.update({k: np.zeros(len(T)) for k in ("U_mean", "U_std", "C_mean", "C_std")})
    st = lib().orc_bootstrap(R, h, W, _ptr(starts), int(e_lo), int(B), _ptr(p), _ptr(v), float(log_total),
                             int(nboot), int(seed), _ptr(T), len(T), float(e_lo if e_first is None else e_first),
                             float(de), _ptr(out["lng_mean"]), _ptr(out["lng_std"]), _ptr(out["U_mean"]),
                             _ptr(out["U_std"]), _ptr(out["C_mean"]), _ptr(out["C_std"]))
    return st, out


def run_pieces(o):
    """(pieces [h, W], visited [h, W]) of a run: walker 0 of every window and the window's flags."""
    pieces = np.stack([o.walker(k * o.m)["lng"] for k in range(o.h)])
    vis = np.stack([o.window(k)["visited"] for k in range(o.h)])
    return pieces, vis


def rep_threshold(p):
    """32-bit threshold of a reptation probability p: a move is a reptation when its word is below it."""
    return min(int(round(p * 2.0**32)), 2**32 - 1)


def log_poly(x):
    return lib().orc_log_poly(float(x))


def obs_thermo(lng, mu, e_first, T, de=1.0):
    """Canonical average of an observable from ln g(E) and its microcanonical mean mu(E)."""
    g = np.ascontiguousarray(lng, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    out = np.zeros_like(T)
    lib().orc_obs_thermo(_ptr(g), _ptr(mu), len(g), float(e_first), float(de), _ptr(T), len(T), _ptr(out))
    return out


def join_pieces(pieces, visited, starts, e_lo, B, log_total):
    pieces = np.ascontiguousarray(pieces, dtype=np.float64)
    vis = np.ascontiguousarray(visited, dtype=np.uint8)
    starts = np.ascontiguousarray(starts, dtype=np.int32)
    h, W = pieces.shape
    out = np.zeros(B)
    cuts = np.zeros(max(h - 1, 1), dtype=np.int32)
    st = lib().orc_join_pieces(h, W, _ptr(starts), e_lo, B, _ptr(pieces), _ptr(vis),
                               float(log_total), _ptr(out), _ptr(cuts))
    return st, out, cuts[: h - 1]


class Rewl:
    """Sequential REWL run over h windows x m walkers of the 2D Potts model."""

    def __init__(self, L, q, windows, overlap, walkers, init_spins, seed=1, instance=0,
                 flat=(4, 5), lnf_init=1.0, lnf_final=1e-6, schedule=0, sync_attempts=1000,
                 exchange=1, precision=0, fixed_lnf=0, shadow=0, walkin_slack=16, obs_bins=0, threads=1):
        self.L, self.q, self.h, self.m = L, q, windows, walkers
        self.precision, self.obs_bins = precision, obs_bins
        spins = np.ascontiguousarray(init_spins, dtype=np.int8).reshape(-1)
        if spins.size != windows * walkers * L * L:
            raise ValueError("init_spins must hold one L*L lattice per walker")
        self._keep = spins
        self.h_ = lib().orc_create(L, q, windows, overlap, walkers, seed, instance, flat[0], flat[1],
                                   lnf_init, lnf_final, schedule, sync_attempts, exchange, precision,
                                   fixed_lnf, shadow, walkin_slack, obs_bins, _ptr(spins))
        if not self.h_:
            raise ValueError("oracle rejected the parameters")
        lib().orc_set_threads(self.h_, threads)
        info = self.info()
        self.N, self.W, self.B, self.e_lo, self.nw = info[:5]
        self.starts = np.zeros(windows, dtype=np.int32)
        lib().orc_starts(self.h_, _ptr(self.starts))

    @classmethod
    def trimer(cls, nmol, box, e_min, bin_w, bins, windows, overlap, walkers, init_coords, seed=1,
               instance=0, flat=(4, 5), lnf_init=1.0, lnf_final=1e-6, schedule=0, sync_attempts=1000,
               exchange=1, precision=0, fixed_lnf=0, shadow=0, walkin_slack=16, threads=1):
        """REWL run of the trimer model; init_coords: float32 [walkers, 3 nmol, 3]."""
        self = cls.__new__(cls)
        self.h, self.m, self.precision, self.nmol = windows, walkers, precision, nmol
        self.obs_bins = 0
        x = np.ascontiguousarray(init_coords, dtype=np.float32).reshape(-1)
        if x.size != windows * walkers * nmol * 9:
            raise ValueError("init_coords must hold 3 nmol beads x 3 coordinates per walker")
        self._keep = x
        self.h_ = lib().orc_create_trimer(nmol, box, e_min, bin_w, bins, windows, overlap, walkers, seed,
                                          instance, flat[0], flat[1], lnf_init, lnf_final, schedule,
                                          sync_attempts, exchange, precision, fixed_lnf, shadow,
                                          walkin_slack, _ptr(x))
        if not self.h_:
            raise ValueError("oracle rejected the parameters")
        lib().orc_set_threads(self.h_, threads)
        info = self.info()
        self.N, self.W, self.B, self.e_lo, self.nw = info[:5]
        self.starts = np.zeros(windows, dtype=np.int32)
        lib().orc_starts(self.h_, _ptr(self.starts))
        return self

    @classmethod
    def lipid(cls, nlip, nsol, box, e_min, bin_w, bins, windows, overlap, walkers, init_coords, eps_ww=1.0,
              rep_prob=None, seed=1, instance=0, flat=(4, 5), lnf_init=1.0, lnf_final=1e-6, schedule=0,
              sync_attempts=1000, exchange=1, fixed_lnf=0, walkin_slack=16, threads=1):
        """REWL run of the lipid model with explicit solvent; init_coords float32 [walkers, np, 3].

        rep_prob: reptation probability per update (default 3 nlip / (10 np))."""
        self = cls.__new__(cls)
        np_ = 3 * nlip + nsol
        self.h, self.m, self.precision, self.nlip, self.np = windows, walkers, 0, nlip, np_
        self.obs_bins = 0
        if rep_prob is None:
            rep_prob = 3.0 * nlip / (10.0 * np_)
        self.rep_thr = rep_threshold(rep_prob)
        x = np.ascontiguousarray(init_coords, dtype=np.float32).reshape(-1)
        if x.size != windows * walkers * np_ * 3:
            raise ValueError("init_coords must hold np particles x 3 coordinates per walker")
        self._keep = x
        self.h_ = lib().orc_create_lipid(nlip, nsol, box, eps_ww, self.rep_thr, e_min, bin_w, bins, windows,
                                         overlap, walkers, seed, instance, flat[0], flat[1], lnf_init, lnf_final,
                                         schedule, sync_attempts, exchange, fixed_lnf, walkin_slack, _ptr(x))
        if not self.h_:
            raise ValueError("oracle rejected the parameters")
        lib().orc_set_threads(self.h_, threads)
        info = self.info()
        self.N, self.W, self.B, self.e_lo, self.nw = info[:5]
        self.starts = np.zeros(windows, dtype=np.int32)
        lib().orc_starts(self.h_, _ptr(self.starts))
        return self

    def lipid_state(self, w):
        """(coords float32 [np, 3], types int8 [np] (0 P, 1 H, 2 W), lipids int32 [nlip, 3])."""
        x = np.zeros((self.np, 3), dtype=np.float32)
        t = np.zeros(self.np, dtype=np.int8)
        lp = np.zeros((self.nlip, 3), dtype=np.int32)
        lib().orc_lipid_state(self.h_, w, _ptr(x), _ptr(t), _ptr(lp))
        return x, t, lp

    def lipid_energy_fx(self, w):
        """Total energy of walker w's configuration recomputed from scratch, in units of 2^-32
        (None for a hard overlap)."""
        e = ctypes.c_int64(0)
        return e.value if lib().orc_lipid_energy_fx(self.h_, w, ctypes.byref(e)) else None

    def lipid_energy(self, w):
        e = self.lipid_energy_fx(w)
        return None if e is None else fx_to_float(e)

    def lipid_delta_move_fx(self, w, b, xn):
        """Energy change of displacing particle b to xn, in units of 2^-32 (None for a hard overlap)."""
        e = ctypes.c_int64(0)
        ok = lib().orc_lipid_delta_move_fx(self.h_, w, b, _ptr(np.ascontiguousarray(xn, dtype=np.float32)),
                                           ctypes.byref(e))
        return e.value if ok else None

    def lipid_delta_move(self, w, b, xn):
        e = self.lipid_delta_move_fx(w, b, xn)
        return None if e is None else fx_to_float(e)

    def lipid_reptate(self, w, lipid, end, pick):
        """Apply a reptation; returns (n_c, n_r, energy change) or None if no solvent is near that end."""
        nc, nr, de = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int64(0)
        if not lib().orc_lipid_reptate(self.h_, w, lipid, end, pick, ctypes.byref(nc), ctypes.byref(nr),
                                       ctypes.byref(de)):
            return None
        return nc.value, nr.value, de.value

    def lipid_pair(self, ti, tj, bonded, r2):
        return lib().orc_lipid_pair(self.h_, ti, tj, bonded, r2)

    def energy(self, w):
        """Current energy of walker w (the continuous models' energy, nearest binary64)."""
        return lib().orc_get_energy(self.h_, w)

    def energy_fx(self, w):
        """Current energy of walker w in units of 2^-32 (continuous models)."""
        return lib().orc_get_energy_fx(self.h_, w)

    def trimer_energy_fx(self, w):
        """Total energy of walker w's configuration recomputed from scratch, in units of 2^-32
        (None for a hard overlap)."""
        e = ctypes.c_int64(0)
        return e.value if lib().orc_trimer_energy_fx(self.h_, w, ctypes.byref(e)) else None

    def trimer_energy(self, w):
        e = self.trimer_energy_fx(w)
        return None if e is None else fx_to_float(e)

    def trimer_delta_fx(self, w, bead, xn):
        """Energy change of moving bead to xn, in units of 2^-32 (None for a hard overlap)."""
        e = ctypes.c_int64(0)
        ok = lib().orc_trimer_delta_fx(self.h_, w, bead, _ptr(np.ascontiguousarray(xn, dtype=np.float32)),
                                       ctypes.byref(e))
        return e.value if ok else None

    def trimer_delta(self, w, bead, xn):
        e = self.trimer_delta_fx(w, bead, xn)
        return None if e is None else fx_to_float(e)

    def __del__(self):
        if getattr(self, "h_", None):
            lib().orc_destroy(self.h_)
            self.h_ = None

    def info(self):
        out = np.zeros(9, dtype=np.int64)
        lib().orc_info(self.h_, _ptr(out))
        return [int(x) for x in out]

    @property
    def step(self):
        return self.info()[5]

    @property
    def round(self):
        return self.info()[6]

    def set_threads(self, n):
        lib().orc_set_threads(self.h_, n)

    def walkin(self, budget=10**9):
        return lib().orc_walkin(self.h_, budget)

    def run(self, attempts, walkin_budget=10**9):
        return lib().orc_run(self.h_, int(attempts), int(walkin_budget))

    def exchange(self):
        return lib().orc_exchange(self.h_)

    def walker(self, w):
        N, W = self.N, self.W
        spins = np.zeros(N, dtype=np.int8)
        E = ctypes.c_int32(0)
        H = np.zeros(W, dtype=np.uint32)
        lng = np.zeros(W)
        hi = np.zeros(W, dtype=np.float32)
        lo = np.zeros(W, dtype=np.float32)
        rep = ctypes.c_uint32(0)
        wa = ctypes.c_int64(0)
        lib().orc_get_walker(self.h_, w, _ptr(spins), ctypes.byref(E), _ptr(H), _ptr(lng),
                             _ptr(hi), _ptr(lo), ctypes.byref(rep), ctypes.byref(wa))
        d = dict(spins=spins, E=E.value, H=H, lng=lng, replica=rep.value, walkin_attempts=wa.value)
        if self.precision == 1:
            d["lng_hi"], d["lng_lo"] = hi, lo
        return d

    def window(self, k):
        lnf, lnf_last = ctypes.c_double(0), ctypes.c_double(0)
        regime, fin = ctypes.c_int32(0), ctypes.c_int32(0)
        it = ctypes.c_int64(0)
        vis = np.zeros(self.W, dtype=np.uint8)
        xa, xc = ctypes.c_uint64(0), ctypes.c_uint64(0)
        lib().orc_get_window(self.h_, k, ctypes.byref(lnf), ctypes.byref(lnf_last), ctypes.byref(regime),
                             ctypes.byref(fin), ctypes.byref(it), _ptr(vis), ctypes.byref(xa),
                             ctypes.byref(xc))
        return dict(lnf=lnf.value, lnf_last=lnf_last.value, regime=regime.value, finished=fin.value,
                    iterations=it.value, visited=vis, x_att=xa.value, x_acc=xc.value)

    def replicas(self):
        """(window_of, trips), uint32 [h*m] by replica id: current window and completed round trips."""
        win = np.zeros(self.nw, dtype=np.uint32)
        trips = np.zeros(self.nw, dtype=np.uint32)
        lib().orc_get_replicas(self.h_, _ptr(win), _ptr(trips))
        return win, trips

    def begin_production(self):
        """Freeze the current ln g as weights (ln f = 0 everywhere), no termination, restart H."""
        return lib().orc_begin_production(self.h_)

    def obs(self, w):
        """Walker w's H(E, O) [W, obs_bins], sum of O [W] and samples [W]."""
        hist = np.zeros((self.W, self.obs_bins), dtype=np.uint32)
        s = np.zeros(self.W, dtype=np.uint64)
        c = np.zeros(self.W, dtype=np.uint32)
        if lib().orc_get_obs(self.h_, w, _ptr(hist), _ptr(s), _ptr(c)) != 0:
            raise ValueError("observable not sampled")
        return hist, s, c

    def obs_micro(self):
        """(mean O [B], samples [B]) pooled over the walkers of every window holding the bin."""
        mean = np.zeros(self.B)
        cnt = np.zeros(self.B, dtype=np.uint64)
        if lib().orc_obs_micro(self.h_, _ptr(mean), _ptr(cnt)) != 0:
            raise ValueError("observable not sampled")
        return mean, cnt

    def replica_visits(self, w):
        """uint32 [h*m]: lookups that found each replica id in walker slot w."""
        out = np.zeros(self.nw, dtype=np.uint32)
        if lib().orc_get_replica_visits(self.h_, w, _ptr(out)) != 0:
            raise ValueError("visit matrix not kept")
        return out

    def shadow(self, w):
        """(hi, lo): double-double exact reference of walker w's ln g."""
        hi, lo = np.zeros(self.W), np.zeros(self.W)
        lib().orc_get_shadow(self.h_, w, _ptr(hi), _ptr(lo))
        return hi, lo

    def set_lng(self, w, lng):
        a = np.ascontiguousarray(lng, dtype=np.float64)
        assert a.size == self.W
        lib().orc_set_lng(self.h_, w, _ptr(a))

    def plant_walker(self, w, H, visited):
        """Overwrite walker w's histogram H [W] and its own visited flags [W]."""
        H = np.ascontiguousarray(H, dtype=np.uint32)
        v = np.ascontiguousarray(visited, dtype=np.uint8)
        assert H.size == self.W and v.size == self.W
        lib().orc_plant_walker(self.h_, w, _ptr(H), _ptr(v))

    def set_step(self, step):
        """Set the main-phase attempts per walker (the t of the 1/t rule is step / W)."""
        lib().orc_set_step(self.h_, int(step))

    def set_window(self, k, lnf, regime=0):
        lib().orc_set_window(self.h_, k, float(lnf), int(regime))

    def sync_window(self, k):
        """Run window k's sync step (flatness, averaging, ln f, termination) on the current state."""
        lib().orc_sync_window(self.h_, k)

    def join(self):
        out = np.zeros(self.B)
        cuts = np.zeros(max(self.h - 1, 1), dtype=np.int32)
        st = lib().orc_join(self.h_, _ptr(out), _ptr(cuts))
        return st, out, cuts[: self.h - 1]
