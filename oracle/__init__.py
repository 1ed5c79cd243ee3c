"""CPU oracle for the DPSNN cortical-grid hot path.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It is a plain, slow C
implementation (oracle/dpsnn_oracle.c, and oracle/dpsnn_waves.c for the
slow-wave analysis of Sec. 2.3) written from the paper and bound here with
ctypes; it shares no code with the HIP library.

Parameters are passed as a plain dict whose keys are the field names of
``orc_params`` (pairs are ``[excitatory, inhibitory]``; the population-model
fields default to the two-population model when absent).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liborc.so")

MIRROR32 = 0
EXACT64 = 1
WEIGHT_DTYPES = {"f32": 0, "f16": 1, "i8": 2}

_PAIR = C.c_double * 2
_I4 = C.c_int32 * 4
_D4 = C.c_double * 4
_I44 = (C.c_int32 * 4) * 4
_D44 = (C.c_double * 4) * 4
# population-model fields and their defaults (two-population model)
_POP_FIELDS = [
    ("n_pops", C.c_int32), ("open_boundary", C.c_int32), ("pop_size", _I4),
    ("pop_exc", _I4), ("n_syn", _I44), ("J_mean_ts", _D44), ("J_sd_ts", _D44),
    ("p_nu_ext_hz", _D4), ("p_Jext_mean", _D4), ("p_Jext_sd", _D4),
    ("p_tau_m", _D4), ("p_E", _D4), ("p_V_th", _D4), ("p_V_r", _D4),
    ("p_tau_arp", _D4), ("p_alpha_c", _D4), ("p_tau_c", _D4), ("p_gc", _D4),
    ("p_I_const", _D4),
]
# plasticity fields (default: off)
_STDP_FIELDS = [
    ("plastic", C.c_int32), ("stdp_update_steps", C.c_int32), ("stdp_A_plus", C.c_double),
    ("stdp_A_minus", C.c_double), ("stdp_tau_plus", C.c_double),
    ("stdp_tau_minus", C.c_double), ("stdp_tau_y", C.c_double), ("stdp_eta", C.c_double),
    ("stdp_w_max", C.c_double),
]


class OrcParams(C.Structure):
    _fields_ = [
        ("grid_w", C.c_int32), ("grid_h", C.c_int32), ("K", C.c_int32),
        ("K_out", C.c_int32), ("frac_exc", C.c_double), ("frac_local", _PAIR),
        ("lambda_", C.c_double), ("torus", C.c_int32), ("d_min", C.c_int32),
        ("d_max", C.c_int32), ("dt_ms", C.c_double), ("weight_dtype", C.c_int32),
        ("acc_bits", C.c_int32), ("q_frac_bits", C.c_int32),
        ("J_mean", _PAIR), ("J_sd", _PAIR), ("nu_ext_hz", _PAIR),
        ("Jext_mean", _PAIR), ("Jext_sd", _PAIR), ("tau_m", _PAIR), ("E", _PAIR),
        ("V_th", _PAIR), ("V_r", _PAIR), ("tau_arp", _PAIR), ("alpha_c", _PAIR),
        ("tau_c", _PAIR), ("gc", _PAIR), ("I_const", _PAIR),
        ("rate_bin_steps", C.c_int32),
    ] + _POP_FIELDS + _STDP_FIELDS


def _fill(ctype, v):
    if ctype in (_I44, _D44):
        out = ctype()
        el = C.c_int32 if ctype is _I44 else C.c_double
        for i in range(4):
            for j in range(4):
                x = v[i][j] if i < len(v) and j < len(v[i]) else 0
                out[i][j] = el(int(x) if el is C.c_int32 else float(x)).value
        return out
    if ctype in (_I4, _D4):
        vals = [v[i] if i < len(v) else 0 for i in range(4)]
        return ctype(*[(int(x) if ctype is _I4 else float(x)) for x in vals])
    return None


def to_struct(params: dict) -> OrcParams:
    s = OrcParams()
    pop_names = {n for n, _ in _POP_FIELDS}
    stdp_names = {n for n, _ in _STDP_FIELDS}
    for name, ctype in OrcParams._fields_:
        key = "lambda" if name == "lambda_" else name
        if key in pop_names and key not in params:
            continue                      # zero: the two-population model
        if key in stdp_names and key not in params:
            continue                      # zero: no plasticity
        if params.get("n_pops", 0) and key not in params:
            continue                      # two-population fields unused
        v = params[key]
        if key == "weight_dtype" and isinstance(v, str):
            v = WEIGHT_DTYPES[v]
        if ctype is _PAIR:
            setattr(s, name, _PAIR(float(v[0]), float(v[1])))
        elif ctype in (_I4, _D4, _I44, _D44):
            setattr(s, name, _fill(ctype, v))
        elif ctype is C.c_double:
            setattr(s, name, float(v))
        else:
            setattr(s, name, int(v))
    return s


class OrcWaveParams(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("n_pops", C.c_int32),
                ("bin_steps", C.c_int32), ("dt_ms", C.c_double), ("bin0", C.c_int64),
                ("noise_var", C.c_double), ("seed", C.c_uint64), ("min_down", C.c_int32),
                ("min_up", C.c_int32), ("min_modules", C.c_int32), ("reserved", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            _build.build()
        L = C.CDLL(_LIBPATH)
        P = C.POINTER
        L.orc_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.orc_philox4x32_10.restype = None
        L.orc_normal_quantile.argtypes = [C.c_double]
        L.orc_normal_quantile.restype = C.c_double
        L.orc_f64_to_f16.argtypes = [C.c_double]
        L.orc_f64_to_f16.restype = C.c_uint16
        L.orc_f16_to_f64.argtypes = [C.c_uint16]
        L.orc_f16_to_f64.restype = C.c_double
        L.orc_create.argtypes = [P(OrcParams), C.c_uint64, C.c_int32, C.c_int32, P(C.c_int32)]
        L.orc_create.restype = C.c_void_p
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_free.restype = None
        for f in ("orc_n_neurons", "orc_time"):
            getattr(L, f).argtypes = [C.c_void_p]
            getattr(L, f).restype = C.c_int64
        for f in ("orc_n_slots", "orc_status"):
            getattr(L, f).argtypes = [C.c_void_p]
            getattr(L, f).restype = C.c_int32
        L.orc_table.argtypes = [C.c_void_p, C.c_char_p, C.c_void_p, C.c_int64]
        L.orc_table.restype = C.c_int64
        L.orc_gen_row.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p]
        L.orc_gen_row.restype = C.c_int32
        L.orc_gen_row_blocks.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_gen_row_blocks.restype = C.c_int32
        L.orc_n_pops.argtypes = [C.c_void_p]
        L.orc_n_pops.restype = C.c_int32
        L.orc_ext_input.argtypes = [C.c_void_p, C.c_int64, C.c_int64,
                                    P(C.c_int64), P(C.c_double)]
        L.orc_ext_input.restype = C.c_int32
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_step.restype = C.c_int32
        L.orc_get_state.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_get_state.restype = C.c_int32
        L.orc_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_set_state.restype = C.c_int32
        L.orc_get_ring.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_get_ring.restype = C.c_int32
        L.orc_set_ring.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_set_ring.restype = C.c_int32
        L.orc_set_time.argtypes = [C.c_void_p, C.c_int64]
        L.orc_set_time.restype = C.c_int32
        L.orc_spikes.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]
        L.orc_spikes.restype = C.c_int64
        L.orc_rates.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
        L.orc_rates.restype = C.c_int64
        L.orc_plasticity.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                     C.c_void_p]
        L.orc_plasticity.restype = C.c_int32
        L.orc_waves.argtypes = [P(OrcWaveParams), C.c_void_p, C.c_int64, C.c_void_p,
                                C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_int64, P(C.c_int64)]
        L.orc_waves.restype = C.c_int64
        L.orc_wave_transitions_max.argtypes = [C.c_int64, C.c_int32, C.c_int32]
        L.orc_wave_transitions_max.restype = C.c_int64
        _lib = L
    return _lib


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def normal_quantile(p: float) -> float:
    return lib().orc_normal_quantile(float(p))


def f64_to_f16_bits(x: float) -> int:
    return int(lib().orc_f64_to_f16(float(x)))


def f16_bits_to_f64(h: int) -> float:
    return float(lib().orc_f16_to_f64(int(h)))


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def waves(counts, W: int, H: int, bin_steps: int, dt_ms: float, bin0: int = 0,
          noise_var: float = 0.5, seed: int = 1, min_down: int = 2, min_up: int = 2,
          min_modules: int = 1) -> dict:
    """Slow-wave analysis (Sec. 2.3, Eq. 4) of counts [bins][W*H][pops]:
    transitions in the order (bin, fraction, module) with module, time (ms)
    and wave; per wave the speed (inter-module distances per second, NaN
    where not measured), first transition time and module count."""
    c = np.ascontiguousarray(counts, dtype=np.uint32)
    nb, M, P = c.shape
    assert M == W * H
    wp = OrcWaveParams(W, H, P, bin_steps, dt_ms, bin0, noise_var, seed, min_down, min_up,
                       min_modules, 0)
    cap = M * lib().orc_wave_transitions_max(nb, min_down, min_up)
    tm = np.zeros(cap, np.int32)
    tT = np.zeros(cap, np.float64)
    tw = np.zeros(cap, np.int32)
    ws = np.zeros(cap, np.float64)
    wt = np.zeros(cap, np.float64)
    wn = np.zeros(cap, np.int32)
    nw = C.c_int64(0)
    n = lib().orc_waves(C.byref(wp), _ptr(c), nb, _ptr(tm), _ptr(tT), _ptr(tw), cap,
                        _ptr(ws), _ptr(wt), _ptr(wn), cap, C.byref(nw))
    if n < 0:
        raise ValueError(f"orc_waves failed ({n})")
    k = nw.value
    return {"module": tm[:n], "T": tT[:n], "wave": tw[:n], "speed": ws[:k], "t0": wt[:k],
            "n": wn[:k]}


class Oracle:
    """One simulated network on the CPU (see oracle/dpsnn_oracle.h)."""

    def __init__(self, params: dict, seed: int, mode: int = MIRROR32,
                 store_rows: bool = True):
        self.params = dict(params)
        self._s = to_struct(params)
        err = C.c_int32(0)
        h = lib().orc_create(C.byref(self._s), C.c_uint64(seed), mode,
                             1 if store_rows else 0, C.byref(err))
        if not h:
            raise ValueError(f"orc_create failed ({err.value})")
        self._h = h
        self.seed = seed
        self.mode = mode
        self.N = int(lib().orc_n_neurons(h))
        self.D = int(lib().orc_n_slots(h))
        self.M = int(params["grid_w"]) * int(params["grid_h"])
        self.n_del = int(params["d_max"]) - int(params["d_min"]) + 1
        self.P = int(lib().orc_n_pops(h))

    def pop_of(self, i: int) -> int:
        """Population of neuron i (module-local index against the ranges)."""
        K = int(self.params["K"])
        if self.params.get("n_pops", 0):
            edges = np.cumsum(self.params["pop_size"][: self.P])
        else:
            edges = [round(self.params["frac_exc"] * K), K]
        return int(np.searchsorted(edges, int(i) % K, side="right"))

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    @property
    def t(self) -> int:
        return int(lib().orc_time(self._h))

    @property
    def status(self) -> int:
        return int(lib().orc_status(self._h))

    def step(self, n: int) -> int:
        return int(lib().orc_step(self._h, int(n)))

    def table(self, name: str, dtype) -> np.ndarray:
        nb = lib().orc_table(self._h, name.encode(), None, 0)
        if nb < 0:
            raise KeyError(name)
        out = np.zeros(nb // np.dtype(dtype).itemsize, dtype=dtype)
        lib().orc_table(self._h, name.encode(), _ptr(out), nb)
        return out

    def gen_row(self, s: int):
        Ko = int(self.params["K_out"])
        tgt = np.zeros(Ko, np.int32)
        dl = np.zeros(Ko, np.uint8)
        wi = np.zeros(Ko, np.uint16)
        doff = np.zeros(self.n_del + 1, np.uint16)
        rc = lib().orc_gen_row(self._h, int(s), _ptr(tgt), _ptr(dl), _ptr(wi), _ptr(doff))
        if rc != 0:
            raise ValueError(rc)
        return tgt, dl, wi, doff

    def gen_row_blocks(self, s: int):
        """(targets, delays, efficacy indices, delay offsets, blocks)."""
        Ko = int(self.params["K_out"])
        tgt = np.zeros(Ko, np.int32)
        dl = np.zeros(Ko, np.uint8)
        wi = np.zeros(Ko, np.uint16)
        bk = np.zeros(Ko, np.uint8)
        doff = np.zeros(self.n_del + 1, np.uint16)
        rc = lib().orc_gen_row_blocks(self._h, int(s), _ptr(tgt), _ptr(dl), _ptr(wi),
                                      _ptr(doff), _ptr(bk))
        if rc != 0:
            raise ValueError(rc)
        return tgt, dl, wi, doff, bk

    def ext_input(self, i: int, t: int):
        fs = C.c_int64(0)
        ds = C.c_double(0.0)
        k = lib().orc_ext_input(self._h, int(i), int(t), C.byref(fs), C.byref(ds))
        return int(k), int(fs.value), float(ds.value)

    def state(self):
        V = np.zeros(self.N)
        c = np.zeros(self.N)
        r = np.zeros(self.N, np.int32)
        lib().orc_get_state(self._h, _ptr(V), _ptr(c), _ptr(r))
        return V, c, r

    def set_state(self, V=None, c=None, ref=None):
        V = None if V is None else np.ascontiguousarray(V, np.float64)
        c = None if c is None else np.ascontiguousarray(c, np.float64)
        ref = None if ref is None else np.ascontiguousarray(ref, np.int32)
        lib().orc_set_state(self._h, _ptr(V), _ptr(c), _ptr(ref))

    def ring(self) -> np.ndarray:
        if self.mode == MIRROR32:
            out = np.zeros(self.D * self.N, np.int64)
            lib().orc_get_ring(self._h, _ptr(out), None)
        else:
            out = np.zeros(self.D * self.N, np.float64)
            lib().orc_get_ring(self._h, None, _ptr(out))
        return out.reshape(self.D, self.N)

    def set_ring(self, ring):
        if self.mode == MIRROR32:
            r = np.ascontiguousarray(ring, np.int64).reshape(-1)
            assert r.size == self.D * self.N
            lib().orc_set_ring(self._h, _ptr(r), None)
        else:
            r = np.ascontiguousarray(ring, np.float64).reshape(-1)
            assert r.size == self.D * self.N
            lib().orc_set_ring(self._h, None, _ptr(r))

    def set_time(self, t: int):
        lib().orc_set_time(self._h, int(t))

    def spikes(self):
        n = lib().orc_spikes(self._h, None, None, 0)
        st = np.zeros(n, np.int32)
        ids = np.zeros(n, np.int32)
        lib().orc_spikes(self._h, _ptr(st), _ptr(ids), n)
        return st, ids

    def rates(self) -> np.ndarray:
        nb = lib().orc_rates(self._h, None, 0)
        out = np.zeros((nb, self.M, self.P), np.uint32)
        lib().orc_rates(self._h, _ptr(out), nb)
        return out

    def plasticity(self, s: int):
        """Row s's last activation steps, signals and efficacies, in the
        order of gen_row_blocks."""
        Ko = int(self.params["K_out"])
        ta = np.zeros(Ko, np.int32)
        y = np.zeros(Ko, np.float64)
        w = np.zeros(Ko, np.float64)
        rc = lib().orc_plasticity(self._h, s, _ptr(ta), _ptr(y), _ptr(w))
        if rc != 0:
            raise ValueError("no plasticity state")
        return ta, y, w
