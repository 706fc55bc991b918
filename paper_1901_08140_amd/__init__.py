"""Python binding of libswarm.so, the MI355X (gfx950) electron-swarm library.

Argument marshalling only: every step of the method (rate tables, null-collision flight,
scattering, secondaries, tallies) runs in the library's HIP kernels.  The function names
are those of the C ABI in include/swarm.h.  PyTorch is used only to hand over a HIP stream
(any object with a `cuda_stream` attribute, or an integer stream handle).

The library must have been built (paper_1901_08140_amd/build.py); importing this module
without it raises ImportError -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libswarm.so")

SWARM_OK, SWARM_ERR_INVALID_ARG, SWARM_ERR_OUT_OF_MEMORY, SWARM_ERR_CAPACITY = 0, -1, -2, -3
SWARM_ERR_DEVICE, SWARM_ERR_STATE, SWARM_PENDING = -4, -5, 1
SWARM_ELASTIC, SWARM_EXCITATION, SWARM_IONIZATION, SWARM_ATTACHMENT = 0, 1, 2, 3
SWARM_FP64, SWARM_FP32_MIXED = 0, 1
SWARM_DUMMY, SWARM_REAL = 0, 1
SWARM_TRIAL_CONSTANT, SWARM_TRIAL_VARIABLE, SWARM_TRIAL_BINNED = 0, 1, 2
SWARM_SCATTER_ISOTROPIC, SWARM_SCATTER_SCREENED_COULOMB, SWARM_SCATTER_CONSTANT_XI = 0, 1, 2
SWARM_SCHEDULE_ALL, SWARM_SCHEDULE_SHORTEST_FIRST = 0, 1

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1901_08140_amd/build.py`")
# torch ships its own HIP and HSA runtimes.  Loading torch first lets the library bind to those
# (same sonames) instead of a second copy from /opt/rocm, which cannot open the device once
# torch's copy holds it.
try:
    import torch  # noqa: F401
except ImportError:
    pass
_lib = ctypes.CDLL(LIB_PATH)

_d, _i32, _i64, _u64, _vp = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
_P = ctypes.POINTER


class swarm_channel(ctypes.Structure):
    _fields_ = [("kind", _i32), ("threshold_eV", _d), ("n_points", _i32),
                ("energy_eV", _P(_d)), ("sigma_m2", _P(_d))]


class swarm_component(ctypes.Structure):
    _fields_ = [("mass_amu", _d), ("fraction", _d), ("n_channels", _i32),
                ("channels", _P(swarm_channel)), ("scattering", _i32), ("mt_over_el", _d)]


class swarm_params(ctypes.Structure):
    _fields_ = [("E_V_per_m", _d), ("B_T", _d), ("B_angle_rad", _d), ("N_per_m3", _d), ("T_K", _d),
                ("init_energy_eV", _d), ("precision", _i32), ("secondaries", _i32),
                ("grid_points_per_octave", _i32), ("grid_min_exp2", _i32), ("grid_max_exp2", _i32),
                ("user_majorant", _d), ("capacity", _i64), ("stream", _vp),
                ("trial_strategy", _i32), ("trial_zeta", _d), ("trial_grace", _i64),
                ("trial_bins", _i32), ("thermal_targets", _i32), ("relativistic", _i32)]


class swarm_stat(ctypes.Structure):
    _fields_ = [("value", _d), ("stat_sigma", _d), ("spread", _d)]


_STAT_NAMES = ["W", "Wx", "Wy", "Wz", "mean_energy", "mean_energy_after", "D", "DL", "DT", "sigma",
               "sigmaL", "sigmaT", "D_vec", "DL_vec", "DT_vec", "sigma_vec", "sigmaL_vec",
               "sigmaT_vec", "alpha", "eta"]
_COUNT_NAMES = ["n_real", "n_null", "n_forbidden", "n_fail", "n_over", "n_electrons", "n_finished",
                "n_attached", "n_stuck", "n_created", "n_ionizations", "n_attachments", "n_dropped"]


class swarm_tallies_t(ctypes.Structure):
    _fields_ = ([(n, swarm_stat) for n in _STAT_NAMES] +
                [("alpha_rate", _d), ("eta_rate", _d), ("efficiency", _d), ("majorant", _d)] +
                [(n, _i64) for n in _COUNT_NAMES] +
                [("n_retry_failed", _i64), ("exact", _i32), ("trial_strategy", _i32)])


class swarm_job(ctypes.Structure):
    _fields_ = [("n_electrons", _i64), ("n_collisions", _i64), ("seed", _u64)]


class swarm_launch_opts(ctypes.Structure):
    _fields_ = [("block_size", _i32), ("chunk", _i32), ("pending_trigger", _i32), ("use_graph", _i32),
                ("service_waves", _i32), ("table_layout", _i32), ("park_lanes", _i32)]


class swarm_server_params(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", _i64), ("precision", _i32), ("quantum_collisions", _i64),
                ("max_active", _i32), ("opts", swarm_launch_opts), ("stream", _vp), ("schedule", _i32)]


class swarm_request_info(ctypes.Structure):
    _fields_ = [("submit_s", _d), ("admit_s", _d), ("done_s", _d), ("n_real", _i64), ("epochs", _i64),
                ("bytes", _i64), ("progress", _i64), ("blocks_per_real", _d)]


class swarm_server_stats_t(ctypes.Structure):
    _fields_ = [("time_s", _d), ("n_submitted", _i64), ("n_pending", _i64), ("n_active", _i64),
                ("n_finished", _i64), ("n_failed", _i64), ("bytes_in_use", _i64), ("work_left", _i64),
                ("work_done", _i64), ("epochs", _i64)]


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

_SIGS = {
    "swarm_create": (_i32, [_P(swarm_component), _i32, _P(swarm_params), _P(_vp)]),
    "swarm_run": (_i32, [_vp, _i64, _i64, _u64]),
    "swarm_run_async": (_i32, [_vp, _i64, _i64, _u64]),
    "swarm_wait": (_i32, [_vp]),
    "swarm_create_in_arena": (_i32, [_P(swarm_component), _i32, _P(swarm_params), _vp, _i64, _P(_vp)]),
    "swarm_arena_bytes": (_i32, [_P(swarm_component), _i32, _P(swarm_params), _i64, _P(_i64)]),
    "swarm_run_noalloc": (_i32, [_vp, _i64, _i64, _u64, _vp]),
    "swarm_set_launch_opts": (_i32, [_vp, _P(swarm_launch_opts)]),
    "swarm_tallies": (_i32, [_vp, _P(swarm_tallies_t)]),
    "swarm_records": (_i32, [_vp, _vp, _i64, _P(_i64)]),
    "swarm_set_trace": (_i32, [_vp, _P(_u64), _i32, _i32]),
    "swarm_trace_events": (_i32, [_vp, _vp, _P(_i32)]),
    "swarm_tables": (_i32, [_vp, _P(_i32), _P(_i32), _P(_d), _P(_d), _P(_d)]),
    "swarm_last_timing": (_i32, [_vp, _P(_d), _P(_d)]),
    "swarm_last_launches": (_i32, [_vp, _P(_i64), _P(_i64)]),
    "swarm_destroy": (None, [_vp]),
    "swarm_strerror": (ctypes.c_char_p, [_i32]),
    "swarm_last_error": (ctypes.c_char_p, []),
    "swarm_batch_create": (_i32, [_P(_vp), _P(swarm_job), _i32, _P(swarm_launch_opts), _P(_vp)]),
    "swarm_batch_launch": (_i32, [_vp]),
    "swarm_batch_wait": (_i32, [_vp, _P(_d)]),
    "swarm_batch_tallies": (_i32, [_vp, _i32, _P(swarm_tallies_t)]),
    "swarm_batch_destroy": (None, [_vp]),
    "swarm_batch_run": (_i32, [_P(_vp), _P(swarm_job), _i32, _P(swarm_launch_opts)]),
    "swarm_autotune": (_i32, [_P(_vp), _P(swarm_job), _i32, _i64, _P(swarm_launch_opts)]),
    "swarm_server_create": (_i32, [_P(swarm_server_params), _P(_vp)]),
    "swarm_server_create_in_arena": (_i32, [_P(swarm_server_params), _vp, _i64, _P(_vp)]),
    "swarm_server_submit": (_i32, [_vp, _P(swarm_component), _i32, _P(swarm_params), _i64, _i64, _u64,
                                   _P(_i64)]),
    "swarm_server_submit_records": (_i32, [_vp, _P(swarm_component), _i32, _P(swarm_params), _i64, _i64, _u64,
                                           _vp, _P(_i64)]),
    "swarm_server_poll": (_i32, [_vp, _i64, _P(swarm_tallies_t), _P(swarm_request_info)]),
    "swarm_server_drain": (_i32, [_vp]),
    "swarm_server_now": (_d, [_vp]),
    "swarm_server_stats": (_i32, [_vp, _P(swarm_server_stats_t)]),
    "swarm_server_destroy": (None, [_vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class SwarmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_lib.swarm_strerror(status).decode()}: {message}")
        self.status = status


def _check(st):
    if st < 0:
        raise SwarmError(st, _lib.swarm_last_error().decode())
    return st


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(int(stream.cuda_stream))
    return ctypes.c_void_p(int(stream))


class _Marshalled:
    """ctypes arrays of the components and channels (kept alive for the call)."""

    def __init__(self, components):
        self.keep = []
        self.comps = (swarm_component * len(components))()
        for ci, c in enumerate(components):
            chs = (swarm_channel * len(c.channels))()
            for j, ch in enumerate(c.channels):
                e = np.ascontiguousarray(ch.energy_eV, dtype=np.float64)
                s = np.ascontiguousarray(ch.sigma_m2, dtype=np.float64)
                self.keep += [e, s]
                chs[j].kind = int(ch.kind)
                chs[j].threshold_eV = float(ch.threshold_eV)
                chs[j].n_points = len(e)
                chs[j].energy_eV = e.ctypes.data_as(_P(_d))
                chs[j].sigma_m2 = s.ctypes.data_as(_P(_d))
            self.keep.append(chs)
            self.comps[ci].mass_amu = float(c.mass_amu)
            self.comps[ci].fraction = float(c.fraction)
            self.comps[ci].n_channels = len(c.channels)
            self.comps[ci].channels = chs
            self.comps[ci].scattering = int(getattr(c, "scattering", 0))
            self.comps[ci].mt_over_el = float(getattr(c, "mt_over_el", 1.0))


def make_params(E_V_per_m, B_T=0.0, B_angle_rad=0.0, N_per_m3=2.5e25, T_K=293.0, init_energy_eV=0.1,
                precision=SWARM_FP64, secondaries=SWARM_DUMMY, grid_points_per_octave=0, grid_min_exp2=0,
                grid_max_exp2=0, user_majorant=0.0, capacity=0, stream=None,
                trial_strategy=0, trial_zeta=0.0, trial_grace=0, trial_bins=0, thermal_targets=0,
                relativistic=0):
    p = swarm_params()
    p.E_V_per_m, p.B_T, p.B_angle_rad, p.N_per_m3, p.T_K = E_V_per_m, B_T, B_angle_rad, N_per_m3, T_K
    p.init_energy_eV, p.precision, p.secondaries = init_energy_eV, int(precision), int(secondaries)
    p.grid_points_per_octave, p.grid_min_exp2, p.grid_max_exp2 = grid_points_per_octave, grid_min_exp2, grid_max_exp2
    p.user_majorant, p.capacity = user_majorant, int(capacity)
    p.stream = _stream_handle(stream)
    p.trial_strategy, p.trial_zeta, p.trial_grace = int(trial_strategy), float(trial_zeta), int(trial_grace)
    p.trial_bins = int(trial_bins)
    p.thermal_targets = int(thermal_targets)
    p.relativistic = int(relativistic)
    return p


def params_from_config(cfg, precision=SWARM_FP64, **kw):
    """swarm_params of a synth.SwarmConfig."""
    kw.setdefault("user_majorant", cfg.user_majorant)
    kw.setdefault("trial_strategy", getattr(cfg, "trial_strategy", 0))
    kw.setdefault("trial_zeta", getattr(cfg, "trial_zeta", 0.0))
    kw.setdefault("trial_grace", getattr(cfg, "trial_grace", 0))
    kw.setdefault("trial_bins", getattr(cfg, "trial_bins", 0))
    kw.setdefault("thermal_targets", getattr(cfg, "thermal_targets", 0))
    kw.setdefault("relativistic", getattr(cfg, "relativistic", 0))
    return make_params(cfg.E_V_per_m, cfg.B_T, cfg.B_angle_rad, cfg.N_per_m3, cfg.T_K, cfg.init_energy_eV,
                       precision, cfg.secondaries, **kw)


def swarm_create(components, params):
    m = _Marshalled(components)
    h = _vp()
    _check(_lib.swarm_create(m.comps, len(components), ctypes.byref(params), ctypes.byref(h)))
    return h


def swarm_create_in_arena(components, params, arena_ptr, arena_bytes):
    """arena_ptr: device address (int) of arena_bytes bytes the caller keeps alive."""
    m = _Marshalled(components)
    h = _vp()
    _check(_lib.swarm_create_in_arena(m.comps, len(components), ctypes.byref(params), _vp(int(arena_ptr)),
                                      int(arena_bytes), ctypes.byref(h)))
    return h


def swarm_arena_bytes(components, params, n_electrons):
    m = _Marshalled(components)
    n = _i64(0)
    _check(_lib.swarm_arena_bytes(m.comps, len(components), ctypes.byref(params), int(n_electrons), ctypes.byref(n)))
    return n.value


def swarm_set_launch_opts(h, opts):
    return _check(_lib.swarm_set_launch_opts(h, ctypes.byref(_opts(opts))))


def swarm_run(h, n_electrons, n_collisions, seed):
    """Returns SWARM_OK, or raises SwarmError (status SWARM_ERR_CAPACITY keeps the results)."""
    return _check(_lib.swarm_run(h, int(n_electrons), int(n_collisions), int(seed)))


def swarm_run_async(h, n_electrons, n_collisions, seed):
    return _check(_lib.swarm_run_async(h, int(n_electrons), int(n_collisions), int(seed)))


def swarm_wait(h):
    """The run's status (raises SwarmError like swarm_run)."""
    return _check(_lib.swarm_wait(h))


def swarm_run_noalloc(h, n_electrons, n_collisions, seed, records_ptr):
    """records_ptr: device address (int) of n_electrons records (104 bytes each)."""
    return _check(_lib.swarm_run_noalloc(h, int(n_electrons), int(n_collisions), int(seed), _vp(int(records_ptr))))


def tallies_to_dict(t):
    out = {n: (getattr(t, n).value, getattr(t, n).stat_sigma, getattr(t, n).spread) for n in _STAT_NAMES}
    for n in ("alpha_rate", "eta_rate", "efficiency", "majorant"):
        out[n] = getattr(t, n)
    for n in _COUNT_NAMES + ["n_retry_failed", "exact", "trial_strategy"]:
        out[n] = int(getattr(t, n))
    return out


def swarm_tallies(h):
    t = swarm_tallies_t()
    _check(_lib.swarm_tallies(h, ctypes.byref(t)))
    return tallies_to_dict(t)


def swarm_records(h):
    n = _i64(0)
    _check(_lib.swarm_records(h, None, 0, ctypes.byref(n)))
    rec = np.zeros(n.value, dtype=RECORD_DTYPE)
    _check(_lib.swarm_records(h, rec.ctypes.data_as(_vp), n.value, ctypes.byref(n)))
    return rec


def swarm_set_trace(h, ids, max_events):
    arr = np.ascontiguousarray(ids, dtype=np.uint64)
    _check(_lib.swarm_set_trace(h, arr.ctypes.data_as(_P(_u64)), len(arr), int(max_events)))
    return (len(arr), int(max_events))


def swarm_trace_events(h, n_ids, max_events):
    ev = np.zeros(n_ids * max_events, dtype=EVENT_DTYPE)
    counts = np.zeros(n_ids, dtype=np.int32)
    _check(_lib.swarm_trace_events(h, ev.ctypes.data_as(_vp), counts.ctypes.data_as(_P(_i32))))
    return ev.reshape(n_ids, max_events), counts


def swarm_tables(h):
    G, nc, maj = _i32(0), _i32(0), _d(0)
    _check(_lib.swarm_tables(h, ctypes.byref(G), ctypes.byref(nc), None, None, ctypes.byref(maj)))
    nodes = np.zeros(G.value)
    cum = np.zeros(G.value * nc.value)
    _check(_lib.swarm_tables(h, None, None, nodes.ctypes.data_as(_P(_d)), cum.ctypes.data_as(_P(_d)), None))
    return nodes, cum.reshape(nc.value, G.value), maj.value


def swarm_last_timing(h):
    k, t = _d(0), _d(0)
    _check(_lib.swarm_last_timing(h, ctypes.byref(k), ctypes.byref(t)))
    return k.value, t.value


def swarm_last_launches(h):
    """(simulation launches, electrons parked between them) of the last run."""
    n, p = _i64(0), _i64(0)
    _check(_lib.swarm_last_launches(h, ctypes.byref(n), ctypes.byref(p)))
    return n.value, p.value


def swarm_destroy(h):
    if h:
        _lib.swarm_destroy(h)


def swarm_strerror(status):
    return _lib.swarm_strerror(status).decode()


def swarm_last_error():
    return _lib.swarm_last_error().decode()


# ---- batches -------------------------------------------------------------------------
def _jobs(jobs):
    arr = (swarm_job * len(jobs))()
    for i, (ne, nc, seed) in enumerate(jobs):
        arr[i].n_electrons, arr[i].n_collisions, arr[i].seed = int(ne), int(nc), int(seed)
    return arr


def _opts(opts):
    o = swarm_launch_opts()
    if opts:
        for k, v in opts.items():
            setattr(o, k, int(v))
    return o


def _handles(hs):
    arr = (_vp * len(hs))()
    for i, h in enumerate(hs):
        arr[i] = h.value if isinstance(h, _vp) else h
    return arr


def swarm_batch_create(handles, jobs, opts=None):
    b = _vp()
    _check(_lib.swarm_batch_create(_handles(handles), _jobs(jobs), len(jobs), ctypes.byref(_opts(opts)),
                                   ctypes.byref(b)))
    return b


def swarm_batch_launch(b):
    return _check(_lib.swarm_batch_launch(b))


def swarm_batch_wait(b):
    ms = _d(0)
    _check(_lib.swarm_batch_wait(b, ctypes.byref(ms)))
    return ms.value


def swarm_batch_tallies(b, i):
    t = swarm_tallies_t()
    _check(_lib.swarm_batch_tallies(b, int(i), ctypes.byref(t)))
    return tallies_to_dict(t)


def swarm_batch_destroy(b):
    if b:
        _lib.swarm_batch_destroy(b)


def swarm_batch_run(handles, jobs, opts=None):
    return _check(_lib.swarm_batch_run(_handles(handles), _jobs(jobs), len(jobs), ctypes.byref(_opts(opts))))


def swarm_autotune(handles, jobs, probe_collisions):
    best = swarm_launch_opts()
    _check(_lib.swarm_autotune(_handles(handles), _jobs(jobs), len(jobs), int(probe_collisions),
                               ctypes.byref(best)))
    return {k: getattr(best, k) for k, _ in swarm_launch_opts._fields_}


# ---- serving -------------------------------------------------------------------------
def swarm_server_create(hbm_budget_bytes, precision=SWARM_FP32_MIXED, quantum_collisions=0, max_active=0,
                        opts=None, stream=None, schedule=0):
    p = swarm_server_params()
    p.hbm_budget_bytes, p.precision = int(hbm_budget_bytes), int(precision)
    p.quantum_collisions, p.max_active = int(quantum_collisions), int(max_active)
    p.schedule = int(schedule)
    p.opts = _opts(opts)
    p.stream = _stream_handle(stream)
    s = _vp()
    _check(_lib.swarm_server_create(ctypes.byref(p), ctypes.byref(s)))
    return s


def swarm_server_create_in_arena(arena_ptr, arena_bytes, hbm_budget_bytes=None, precision=SWARM_FP32_MIXED,
                                 quantum_collisions=0, max_active=0, opts=None, stream=None, schedule=0):
    p = swarm_server_params()
    p.hbm_budget_bytes = int(hbm_budget_bytes if hbm_budget_bytes is not None else arena_bytes)
    p.precision = int(precision)
    p.quantum_collisions, p.max_active = int(quantum_collisions), int(max_active)
    p.schedule = int(schedule)
    p.opts = _opts(opts)
    p.stream = _stream_handle(stream)
    s = _vp()
    _check(_lib.swarm_server_create_in_arena(ctypes.byref(p), _vp(int(arena_ptr)), int(arena_bytes), ctypes.byref(s)))
    return s


def swarm_server_submit(s, components, params, n_electrons, n_collisions, seed):
    m = _Marshalled(components)
    t = _i64(0)
    _check(_lib.swarm_server_submit(s, m.comps, len(components), ctypes.byref(params), int(n_electrons),
                                    int(n_collisions), int(seed), ctypes.byref(t)))
    return t.value


def swarm_server_submit_records(s, components, params, n_electrons, n_collisions, seed):
    """(ticket, records array): the array is filled when the request finishes; keep it alive."""
    m = _Marshalled(components)
    rec = np.zeros(int(n_electrons), dtype=RECORD_DTYPE)
    t = _i64(0)
    _check(_lib.swarm_server_submit_records(s, m.comps, len(components), ctypes.byref(params), int(n_electrons),
                                            int(n_collisions), int(seed), rec.ctypes.data_as(_vp), ctypes.byref(t)))
    return t.value, rec


def swarm_server_poll(s, ticket):
    """(done, tallies or None, info dict)."""
    t = swarm_tallies_t()
    info = swarm_request_info()
    st = _check(_lib.swarm_server_poll(s, int(ticket), ctypes.byref(t), ctypes.byref(info)))
    inf = {k: getattr(info, k) for k, _ in swarm_request_info._fields_}
    if st == SWARM_PENDING:
        return False, None, inf
    return True, tallies_to_dict(t), inf


def swarm_server_drain(s):
    return _check(_lib.swarm_server_drain(s))


def swarm_server_stats(s):
    t = swarm_server_stats_t()
    _check(_lib.swarm_server_stats(s, ctypes.byref(t)))
    return {k: getattr(t, k) for k, _ in swarm_server_stats_t._fields_}


def swarm_server_now(s):
    return _lib.swarm_server_now(s)


def swarm_server_destroy(s):
    if s:
        _lib.swarm_server_destroy(s)


# ---- convenience ------------------------------------------------------------------------
class Swarm:
    """Owning wrapper of a swarm handle: Swarm(config, precision).run(n_e, n_c, seed)."""

    def __init__(self, components, params, arena=None):
        """arena: optional (device address, bytes) the handle takes all its device memory from."""
        self.h = swarm_create(components, params) if arena is None else swarm_create_in_arena(components, params,
                                                                                               *arena)

    @classmethod
    def from_config(cls, cfg, precision=SWARM_FP64, arena=None, **kw):
        return cls(cfg.components, params_from_config(cfg, precision, **kw), arena)

    def run(self, n_electrons, n_collisions, seed):
        return swarm_run(self.h, n_electrons, n_collisions, seed)

    def run_async(self, n_electrons, n_collisions, seed):
        return swarm_run_async(self.h, n_electrons, n_collisions, seed)

    def wait(self):
        return swarm_wait(self.h)

    def set_launch_opts(self, opts):
        return swarm_set_launch_opts(self.h, opts)

    def tallies(self):
        return swarm_tallies(self.h)

    def records(self):
        return swarm_records(self.h)

    def tables(self):
        return swarm_tables(self.h)

    def timing(self):
        return swarm_last_timing(self.h)

    def launches(self):
        return swarm_last_launches(self.h)

    def set_trace(self, ids, max_events):
        self._trace = swarm_set_trace(self.h, ids, max_events)

    def trace_events(self):
        return swarm_trace_events(self.h, *self._trace)

    def close(self):
        if self.h:
            swarm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
