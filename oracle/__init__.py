"""FP64 CPU oracle of the null-collision electron-swarm method (Betaboltz, arXiv 1901.08140).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the benchmark's CPU
baseline.  It shares no code with the HIP path (paper_1901_08140_amd); both read their
inputs from the `synth` package, which holds no method arithmetic.

`OracleModel` wraps oracle.cpp (the per-electron simulation); `oracle.tallies` turns its
records into swarm tallies with the paper's estimators.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

RECORD_DTYPE = np.dtype({
    "names": ["id", "flags", "k_start", "k_end", "G", "D", "n_forbidden", "n_over", "n_fail",
              "n_null", "blocks", "r", "t", "sum_eps", "sum_epsp"],
    "formats": ["<u8", "<u4", "<u4", "<u4", "<u4", "<u4", "<u4", "<u4", "<u4",
                "<u8", "<u8", ("<f8", (3,)), "<f8", "<f8", "<f8"],
    "offsets": [0, 8, 12, 16, 20, 24, 28, 32, 36, 40, 48, 56, 80, 88, 96],
    "itemsize": 104,
})
EVENT_DTYPE = np.dtype({
    "names": ["id", "type", "channel", "k", "block", "sub", "pad", "eps", "epsp", "t", "r"],
    "formats": ["<u8", "<i4", "<i4", "<u4", "<u4", "<u4", "<u4", "<f8", "<f8", "<f8", ("<f8", (3,))],
    "offsets": [0, 8, 12, 16, 20, 24, 28, 32, 40, 48, 56],
    "itemsize": 80,
})
FLAG_FINISHED, FLAG_ATTACHED, FLAG_STUCK, FLAG_RETRY_FAILED = 1, 2, 4, 16
EV_REAL, EV_FORBIDDEN, EV_FAIL = 1, 2, 3
CONSTANT_TRIAL, VARIABLE_TRIAL, BINNED_TRIAL = 0, 1, 2
TRIAL_HI, TRIAL_LO, SCAT_HI, SCAT_LO, INIT_HI, INIT_LO, CHILD_ID, THERMAL_HI, THERMAL_LO = range(9)


class _Channel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("threshold_eV", ctypes.c_double),
                ("n_points", ctypes.c_int32), ("energy_eV", ctypes.POINTER(ctypes.c_double)),
                ("sigma_m2", ctypes.POINTER(ctypes.c_double))]


class _Component(ctypes.Structure):
    _fields_ = [("mass_amu", ctypes.c_double), ("fraction", ctypes.c_double),
                ("n_channels", ctypes.c_int32), ("channels", ctypes.POINTER(_Channel)),
                ("scattering", ctypes.c_int32), ("mt_over_el", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("E_V_per_m", ctypes.c_double), ("B_T", ctypes.c_double),
                ("B_angle_rad", ctypes.c_double), ("N_per_m3", ctypes.c_double),
                ("T_K", ctypes.c_double), ("init_energy_eV", ctypes.c_double),
                ("secondaries", ctypes.c_int32), ("grid_P", ctypes.c_int32),
                ("grid_emin", ctypes.c_int32), ("grid_emax", ctypes.c_int32),
                ("user_majorant", ctypes.c_double), ("trial_strategy", ctypes.c_int32),
                ("trial_zeta", ctypes.c_double), ("trial_grace", ctypes.c_int64),
                ("trial_bins", ctypes.c_int32), ("thermal_targets", ctypes.c_int32),
                ("relativistic", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        vp, d, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.c_double, ctypes.c_int32,
                                     ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64)
        P = ctypes.POINTER
        sig = {
            "or_philox": (None, [P(u32), P(u32), P(u32)]),
            "or_stream_block": (None, [u64, u64, u32, u32, P(u32)]),
            "or_uniform53": (d, [u32, u32]),
            "or_create": (vp, [P(_Component), i32, P(_Params), P(i32)]),
            "or_destroy": (None, [vp]),
            "or_n_channels": (i32, [vp]),
            "or_grid_size": (i32, [vp]),
            "or_majorant": (d, [vp]),
            "or_bins": (i32, [vp, P(i32), P(d)]),
            "or_tables": (None, [vp, P(d), P(d)]),
            "or_sigma_raw": (d, [vp, i32, d]),
            "or_rate_raw_total": (d, [vp, d]),
            "or_nu_grid": (d, [vp, d, P(i32)]),
            "or_channel_cum": (d, [vp, i32, d]),
            "or_select": (i32, [vp, d, d]),
            "or_move": (None, [vp, P(d), P(d), d, P(d), P(d)]),
            "or_energy_after": (d, [i32, d, d, d, d]),
            "or_kinetic": (d, [vp, P(d)]),
            "or_speed": (d, [vp, d, i32]),
            "or_const": (d, [i32]),
            "or_xi_from_ratio": (d, [d]),
            "or_target_velocity": (None, [d, P(d), P(d)]),
            "or_moving_target": (i32, [P(d), P(d), d, d, P(d), P(d)]),
            "or_mt_over_el_of_xi": (d, [d]),
            "or_scatter_cos": (d, [i32, d, d, d]),
            "or_rotate": (None, [P(d), d, d, P(d)]),
            "or_run": (vp, [vp, i64, i64, u64, i32, i64, P(u64), i32, i32, i64]),
            "or_run_status": (i32, [vp]),
            "or_run_count": (i64, [vp]),
            "or_run_event_count": (i64, [vp]),
            "or_record_size": (i32, []),
            "or_event_size": (i32, []),
            "or_run_copy": (None, [vp, vp]),
            "or_run_copy_events": (None, [vp, vp]),
            "or_run_free": (None, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        assert L.or_record_size() == RECORD_DTYPE.itemsize
        assert L.or_event_size() == EVENT_DTYPE.itemsize
        _lib = L
    return _lib


def constants():
    L = lib()
    return L.or_const(0), L.or_const(1), L.or_const(2)


def philox(ctr, key):
    L = lib()
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xffffffff for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xffffffff for x in key])
    o = (ctypes.c_uint32 * 4)()
    L.or_philox(c, k, o)
    return [int(x) for x in o]


def stream_block(seed, eid, tag, block):
    o = (ctypes.c_uint32 * 4)()
    lib().or_stream_block(seed, eid, tag, block, o)
    return [int(x) for x in o]


def uniform53(hi, lo):
    return lib().or_uniform53(hi, lo)


def energy_after(kind, eps, eps_k, cos_t, mass_amu):
    return lib().or_energy_after(kind, eps, eps_k, cos_t, mass_amu)


ISOTROPIC, SCREENED_COULOMB, CONSTANT_XI = 0, 1, 2


def boltzmann():
    return lib().or_const(4)


def light_speed():
    return lib().or_const(5)


def target_velocity(sigma, u):
    """Velocity of a moving target: three normals of spread sigma from four uniforms."""
    P = ctypes.POINTER(ctypes.c_double)
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(3)
    lib().or_target_velocity(sigma, u.ctypes.data_as(P), out.ctypes.data_as(P))
    return out


def moving_target(V1, V2, mass_amu, eps_k_eV, u_hat):
    """Electron velocity after a collision with a target moving at V2 (None if forbidden)."""
    P = ctypes.POINTER(ctypes.c_double)
    a, b, h = (np.ascontiguousarray(x, dtype=np.float64) for x in (V1, V2, u_hat))
    out = np.zeros(3)
    ok = lib().or_moving_target(a.ctypes.data_as(P), b.ctypes.data_as(P), mass_amu, eps_k_eV,
                                h.ctypes.data_as(P), out.ctypes.data_as(P))
    return out if ok else None


def hartree_eV():
    return lib().or_const(3)


def xi_from_ratio(r):
    return lib().or_xi_from_ratio(r)


def mt_over_el_of_xi(xi):
    return lib().or_mt_over_el_of_xi(xi)


def scatter_cos(scattering, xi, eps_eV, u):
    return lib().or_scatter_cos(scattering, xi, eps_eV, u)


def rotate(d, cos_t, phi):
    P = ctypes.POINTER(ctypes.c_double)
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.zeros(3)
    lib().or_rotate(d.ctypes.data_as(P), cos_t, phi, out.ctypes.data_as(P))
    return out


class OracleRun:
    def __init__(self, records, events, status):
        self.records = records
        self.events = events
        self.status = status


class OracleModel:
    """A gas mixture in fields E and B, resampled on the octave grid, ready to simulate.

    `components` is a list of synth.Component; field/gas parameters as in synth.SwarmConfig.
    """

    def __init__(self, components, E_V_per_m, B_T=0.0, B_angle_rad=0.0, N_per_m3=2.5e25,
                 T_K=293.0, init_energy_eV=0.1, secondaries=0, grid_P=64, grid_emin=-14,
                 grid_emax=12, user_majorant=0.0, trial_strategy=0, trial_zeta=0.25,
                 trial_grace=5000, trial_bins=10, thermal_targets=0, relativistic=0):
        L = lib()
        self._keep = []
        comps = (_Component * len(components))()
        self.channel_info = []
        for ci, c in enumerate(components):
            chs = (_Channel * len(c.channels))()
            for j, ch in enumerate(c.channels):
                e = np.ascontiguousarray(ch.energy_eV, dtype=np.float64)
                s = np.ascontiguousarray(ch.sigma_m2, dtype=np.float64)
                self._keep += [e, s]
                chs[j].kind = ch.kind
                chs[j].threshold_eV = ch.threshold_eV
                chs[j].n_points = len(e)
                chs[j].energy_eV = e.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                chs[j].sigma_m2 = s.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                self.channel_info.append((ci, ch.kind, ch.threshold_eV, c.mass_amu))
            self._keep.append(chs)
            comps[ci].mass_amu = c.mass_amu
            comps[ci].fraction = c.fraction
            comps[ci].n_channels = len(c.channels)
            comps[ci].channels = chs
            comps[ci].scattering = int(getattr(c, "scattering", 0))
            comps[ci].mt_over_el = float(getattr(c, "mt_over_el", 1.0))
        p = _Params(E_V_per_m, B_T, B_angle_rad, N_per_m3, T_K, init_energy_eV, secondaries,
                    grid_P, grid_emin, grid_emax, user_majorant, trial_strategy, trial_zeta,
                    trial_grace, trial_bins, thermal_targets, relativistic)
        st = ctypes.c_int32(0)
        self.h = L.or_create(comps, len(components), ctypes.byref(p), ctypes.byref(st))
        if not self.h:
            raise ValueError(f"oracle refused the model (status {st.value})")
        self.params = dict(E_V_per_m=E_V_per_m, B_T=B_T, B_angle_rad=B_angle_rad,
                           N_per_m3=N_per_m3, secondaries=secondaries)

    @classmethod
    def from_config(cls, cfg, **kw):
        kw.setdefault("user_majorant", cfg.user_majorant)
        kw.setdefault("trial_strategy", cfg.trial_strategy)
        kw.setdefault("trial_zeta", cfg.trial_zeta)
        kw.setdefault("trial_grace", cfg.trial_grace)
        kw.setdefault("trial_bins", cfg.trial_bins)
        kw.setdefault("thermal_targets", cfg.thermal_targets)
        kw.setdefault("relativistic", cfg.relativistic)
        return cls(cfg.components, cfg.E_V_per_m, cfg.B_T, cfg.B_angle_rad, cfg.N_per_m3, cfg.T_K,
                   cfg.init_energy_eV, cfg.secondaries, **kw)

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_destroy(self.h)
            self.h = None

    # ---- tables -------------------------------------------------------------------------
    @property
    def n_channels(self):
        return lib().or_n_channels(self.h)

    @property
    def grid_size(self):
        return lib().or_grid_size(self.h)

    @property
    def majorant(self):
        return lib().or_majorant(self.h)

    def bins(self):
        """Binned strategy: (bin of every grid node, nu' of every bin)."""
        n = lib().or_bins(self.h, None, None)
        node_bin = np.zeros(self.grid_size if n else 0, dtype=np.int32)
        nup = np.zeros(n)
        if n:
            lib().or_bins(self.h, node_bin.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          nup.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return node_bin, nup

    def tables(self):
        G, nc = self.grid_size, self.n_channels
        nodes = np.zeros(G)
        C = np.zeros(nc * G)
        P = ctypes.POINTER(ctypes.c_double)
        lib().or_tables(self.h, nodes.ctypes.data_as(P), C.ctypes.data_as(P))
        return nodes, C.reshape(nc, G)

    def sigma_raw(self, channel, eps):
        return lib().or_sigma_raw(self.h, channel, eps)

    def rate_raw_total(self, eps):
        return lib().or_rate_raw_total(self.h, eps)

    def nu_grid(self, eps):
        ov = ctypes.c_int32(0)
        v = lib().or_nu_grid(self.h, eps, ctypes.byref(ov))
        return v, bool(ov.value)

    def kinetic(self, u):
        """Kinetic energy (eV) of a held velocity (the proper velocity u = gamma v for the
        relativistic mover)."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        return lib().or_kinetic(self.h, u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))

    def speed(self, eps, proper=False):
        return lib().or_speed(self.h, eps, int(proper))

    def channel_cum(self, c, eps):
        return lib().or_channel_cum(self.h, c, eps)

    def select(self, eps, x):
        return lib().or_select(self.h, eps, x)

    def move(self, r0, v0, T):
        P = ctypes.POINTER(ctypes.c_double)
        r0 = np.ascontiguousarray(r0, dtype=np.float64)
        v0 = np.ascontiguousarray(v0, dtype=np.float64)
        r = np.zeros(3)
        v = np.zeros(3)
        lib().or_move(self.h, r0.ctypes.data_as(P), v0.ctypes.data_as(P), T, r.ctypes.data_as(P),
                      v.ctypes.data_as(P))
        return r, v

    # ---- simulation ---------------------------------------------------------------------
    def run(self, n_electrons, n_collisions, seed, n_threads=None, capacity=0, trace_ids=None,
            max_events=0, first_id=0):
        L = lib()
        if n_threads is None:
            n_threads = max(1, len(os.sched_getaffinity(0)))
        tids = np.ascontiguousarray(trace_ids if trace_ids is not None else [], dtype=np.uint64)
        r = L.or_run(self.h, int(n_electrons), int(n_collisions), int(seed), int(n_threads),
                     int(capacity), tids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                     len(tids), int(max_events), int(first_id))
        try:
            n = L.or_run_count(r)
            rec = np.zeros(n, dtype=RECORD_DTYPE)
            if n:
                L.or_run_copy(r, rec.ctypes.data)
            ne = L.or_run_event_count(r)
            ev = np.zeros(ne, dtype=EVENT_DTYPE)
            if ne:
                L.or_run_copy_events(r, ev.ctypes.data)
            st = L.or_run_status(r)
        finally:
            L.or_run_free(r)
        return OracleRun(rec, ev, st)
