"""Python binding of libdpsnn (include/dpsnn.h): argument marshalling only.

Every step of the simulation runs in the library's HIP kernels; this module
converts parameter dicts to the C struct, passes PyTorch's current HIP
stream and (optionally) PyTorch's caching allocator to the library, and
copies results into NumPy arrays.  There is no fallback: if libdpsnn.so is
missing the import of the library fails loudly.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libdpsnn.so")

ABI_VERSION = 3
W_F32, W_F16, W_I8 = 0, 1, 2
WEIGHT_DTYPES = {"f32": W_F32, "f16": W_F16, "i8": W_I8}
ERRORS = {0: "OK", -1: "INVAL", -2: "NOMEM", -3: "DEVICE", -4: "RANGE",
          -5: "SPIKELOG_FULL", -6: "STATE", -7: "RATES_FULL", -8: "SCRATCH"}

_PAIR = C.c_double * 2
_I4 = C.c_int32 * 4
_D4 = C.c_double * 4
_I44 = (C.c_int32 * 4) * 4
_D44 = (C.c_double * 4) * 4
# population-model fields (zero = the two-population model)
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


class DpsnnParams(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("grid_w", C.c_int32), ("grid_h", C.c_int32),
        ("K", C.c_int32), ("K_out", C.c_int32), ("frac_exc", C.c_double),
        ("frac_local", _PAIR), ("lambda_", C.c_double), ("torus", C.c_int32),
        ("d_min", C.c_int32), ("d_max", C.c_int32), ("dt_ms", C.c_double),
        ("weight_dtype", C.c_int32), ("acc_bits", C.c_int32), ("q_frac_bits", C.c_int32),
        ("J_mean", _PAIR), ("J_sd", _PAIR), ("nu_ext_hz", _PAIR), ("Jext_mean", _PAIR),
        ("Jext_sd", _PAIR), ("tau_m", _PAIR), ("E", _PAIR), ("V_th", _PAIR),
        ("V_r", _PAIR), ("tau_arp", _PAIR), ("alpha_c", _PAIR), ("tau_c", _PAIR),
        ("gc", _PAIR), ("I_const", _PAIR), ("rate_bin_steps", C.c_int32),
        ("spike_log_cap", C.c_int64), ("rate_bins_cap", C.c_int64),
        ("queue_cap", C.c_int32),
    ] + _POP_FIELDS + _STDP_FIELDS


class DpsnnStats(C.Structure):
    _fields_ = [
        ("t", C.c_int64), ("n_neurons", C.c_int64), ("n_modules", C.c_int64),
        ("n_synapses", C.c_int64), ("n_spikes", C.c_int64), ("n_events", C.c_int64),
        ("build_ms", C.c_double), ("bytes_rows", C.c_int64), ("bytes_state", C.c_int64),
        ("bytes_total", C.c_int64), ("lds_bytes", C.c_int32), ("schedule", C.c_int32),
        ("n_index", C.c_int64), ("n_nets", C.c_int32), ("queue_cap", C.c_int32),
        ("deliver_blocks", C.c_int32), ("route_blocks", C.c_int32),
        ("n_pops", C.c_int32), ("queue_entry_bytes", C.c_int32), ("spike_lists", C.c_int32),
    ]


class DpsnnWaveParams(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("net", C.c_int32), ("n_bins", C.c_int64),
        ("noise_var", C.c_double), ("seed", C.c_uint64), ("min_down", C.c_int32),
        ("min_up", C.c_int32), ("min_modules", C.c_int32), ("reserved", C.c_int32),
    ]


class DpsnnWaveResult(C.Structure):
    _fields_ = [
        ("bin0", C.c_int64), ("n_bins", C.c_int64), ("n_transitions", C.c_int64),
        ("n_waves", C.c_int64), ("mean_speed", C.c_double), ("reserved", C.c_double * 3),
    ]


DEFAULT_SPIKE_LOG_CAP = 1 << 24
DEFAULT_RATE_BINS_CAP = 4096


def _fill(ctype, v):
    if ctype in (_I44, _D44):
        out = ctype()
        for i in range(4):
            for j in range(4):
                x = v[i][j] if i < len(v) and j < len(v[i]) else 0
                out[i][j] = int(x) if ctype is _I44 else float(x)
        return out
    vals = [v[i] if i < len(v) else 0 for i in range(4)]
    return ctype(*[(int(x) if ctype is _I4 else float(x)) for x in vals])


def to_struct(params: dict) -> DpsnnParams:
    s = DpsnnParams()
    s.abi_version = ABI_VERSION
    pop_names = {n for n, _ in _POP_FIELDS}
    stdp_names = {n for n, _ in _STDP_FIELDS}
    for name, ctype in DpsnnParams._fields_:
        if name == "abi_version":
            continue
        key = "lambda" if name == "lambda_" else name
        if key in pop_names and key not in params:
            continue                      # zero: the two-population model
        if key in stdp_names and key not in params:
            continue                      # zero: no plasticity
        if params.get("n_pops", 0) and key not in params and key not in (
                "spike_log_cap", "rate_bins_cap", "queue_cap"):
            continue                      # two-population fields unused
        if key == "spike_log_cap":
            v = params.get(key, DEFAULT_SPIKE_LOG_CAP)
        elif key == "rate_bins_cap":
            v = params.get(key, DEFAULT_RATE_BINS_CAP)
        elif key == "queue_cap":
            v = params.get(key, 0)
        else:
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


class DpsnnError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} failed: {ERRORS.get(code, code)} ({code})")
        self.code = code


_lib = None
_ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


def lib():
    """The loaded libdpsnn.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"{LIBPATH} is missing: build it with "
                              "paper_1902_08410_amd.build.build()")
        L = C.CDLL(LIBPATH)
        P, V = C.POINTER, C.c_void_p
        sig = {
            "dpsnn_set_allocator": ([_ALLOC, _FREE, V], C.c_int),
            "dpsnn_build": ([P(DpsnnParams), C.c_uint64, P(V)], C.c_int),
            "dpsnn_set_stream": ([V, V], C.c_int),
            "dpsnn_step": ([V, C.c_int64], C.c_int),
            "dpsnn_sync": ([V], C.c_int),
            "dpsnn_read_spikes": ([V, V, V, C.c_int64, P(C.c_int64)], C.c_int),
            "dpsnn_read_rates": ([V, V, C.c_int64, P(C.c_int64)], C.c_int),
            "dpsnn_stats": ([V, P(DpsnnStats)], C.c_int),
            "dpsnn_stats_get": ([V, P(DpsnnStats)], C.c_int),
            "dpsnn_read_spikes_net": ([V, C.c_int32, V, V, C.c_int64, P(C.c_int64)], C.c_int),
            "dpsnn_read_rates_net": ([V, C.c_int32, V, C.c_int64, P(C.c_int64)], C.c_int),
            "dpsnn_set_routing": ([V, C.c_int32], C.c_int),
            "dpsnn_read_log": ([V, V, V, C.c_int64, P(C.c_int64)], C.c_int),
            "dpsnn_free": ([V], None),
            "dpsnn_strerror": ([C.c_int], C.c_char_p),
            "dpsnn_read_state": ([V, V, V, V], C.c_int),
            "dpsnn_write_state": ([V, V, V, V], C.c_int),
            "dpsnn_read_slots": ([V, V], C.c_int),
            "dpsnn_read_rows": ([V, C.c_int64, C.c_int64, V, V, V], C.c_int),
            "dpsnn_host_table": ([P(DpsnnParams), C.c_char_p, V, C.c_int64], C.c_int64),
            "dpsnn_set_schedule": ([V, C.c_int32], C.c_int),
            "dpsnn_set_graph_steps": ([V, C.c_int64], C.c_int),
            "dpsnn_set_delivery": ([V, C.c_int32, C.c_int32], C.c_int),
            "dpsnn_autotune": ([V, C.c_int64, P(C.c_int32)], C.c_int),
            "dpsnn_profile_steps": ([V, C.c_int64, V], C.c_int),
            "dpsnn_build_batch": ([P(DpsnnParams), P(C.c_uint64), C.c_int32, P(V)], C.c_int),
            "dpsnn_net_info": ([V, C.c_int32, P(C.c_int64), P(C.c_int64), P(C.c_int64),
                                P(C.c_int64)], C.c_int),
            "dpsnn_read_plasticity": ([V, C.c_int64, C.c_int64, V, V], C.c_int),
            "dpsnn_waves": ([V, P(DpsnnWaveParams), P(DpsnnWaveResult), V, V, V, C.c_int64,
                             V, V, V, C.c_int64], C.c_int),
            "dpsnn_waves_counts": ([V, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                    C.c_double, C.c_int64, P(DpsnnWaveParams), V,
                                    P(DpsnnWaveResult), V, V, V, C.c_int64, V, V, V,
                                    C.c_int64], C.c_int),
            "dpsnn_waves_counts_static": ([V, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                           C.c_int32, C.c_double, C.c_int64,
                                           P(DpsnnWaveParams), V, P(DpsnnWaveResult), V, V,
                                           V, C.c_int64, V, V, V, C.c_int64], C.c_int),
        }
        for fn, (args, res) in sig.items():
            f = getattr(L, fn)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


EXPORTS = ["dpsnn_set_allocator", "dpsnn_build", "dpsnn_set_stream", "dpsnn_step",
           "dpsnn_sync", "dpsnn_read_spikes", "dpsnn_read_rates", "dpsnn_stats_get",
           "dpsnn_free", "dpsnn_strerror", "dpsnn_read_state", "dpsnn_write_state",
           "dpsnn_read_slots", "dpsnn_read_rows", "dpsnn_host_table", "dpsnn_set_schedule",
           "dpsnn_set_graph_steps", "dpsnn_autotune", "dpsnn_profile_steps",
           "dpsnn_build_batch", "dpsnn_net_info", "dpsnn_waves", "dpsnn_waves_counts",
           "dpsnn_read_plasticity", "dpsnn_set_delivery", "dpsnn_stats",
           "dpsnn_read_spikes_net", "dpsnn_read_rates_net", "dpsnn_set_routing",
           "dpsnn_waves_counts_static", "dpsnn_read_log"]
SCHED_FUSED, SCHED_SPLIT = 0, 1


def _check(fn, rc):
    if rc != 0:
        raise DpsnnError(fn, rc)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ---- torch as device-memory and stream provider --------------------------
class _TorchAllocator:
    def __init__(self):
        import torch
        self.torch = torch
        self.live = {}
        self.alloc_cb = _ALLOC(self._alloc)
        self.free_cb = _FREE(self._free)

    def _alloc(self, nbytes, ctx):
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device="cuda")
        except Exception:
            return None
        p = t.data_ptr()
        self.live[p] = t
        return p

    def _free(self, ptr, ctx):
        self.live.pop(int(ptr) if ptr else 0, None)


_torch_alloc = None


def use_torch_allocator(enable: bool = True):
    """Route later builds' device allocations through torch's allocator."""
    global _torch_alloc
    if enable:
        if _torch_alloc is None:
            _torch_alloc = _TorchAllocator()
        _check("dpsnn_set_allocator",
               lib().dpsnn_set_allocator(_torch_alloc.alloc_cb, _torch_alloc.free_cb, None))
    else:
        _check("dpsnn_set_allocator", lib().dpsnn_set_allocator(
            C.cast(None, _ALLOC), C.cast(None, _FREE), None))


def current_torch_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


class Net:
    """A built handle (one network, or a batch of networks)."""

    def __init__(self, handle, params, seed):
        self.h = handle
        plist = params if isinstance(params, (list, tuple)) else [params]
        self.params_list = [dict(p) for p in plist]
        self.params = self.params_list[0]
        self.seeds = list(seed) if isinstance(seed, (list, tuple)) else [seed]
        self.seed = self.seeds[0]
        st = self.stats()
        self.n_neurons = int(st["n_neurons"])
        self.N = int(st["n_index"])          # entries of the inspection arrays
        self.M = int(st["n_modules"])
        self.n_nets = int(st["n_nets"])
        self.n_pops = int(st["n_pops"])
        self.D = int(self.params["d_max"]) + 1
        self.n_del = int(self.params["d_max"]) - int(self.params["d_min"]) + 1

    def stats(self) -> dict:
        return dpsnn_stats(self)

    def close(self):
        if self.h:
            lib().dpsnn_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dpsnn_build(params: dict, seed: int, stream=None, torch_memory: bool = True) -> Net:
    if torch_memory:
        use_torch_allocator(True)
    s = to_struct(params)
    h = C.c_void_p()
    _check("dpsnn_build", lib().dpsnn_build(C.byref(s), C.c_uint64(seed), C.byref(h)))
    net = Net(h, params, seed)
    dpsnn_set_stream(net, current_torch_stream() if stream is None else stream)
    return net


def dpsnn_build_batch(params_list, seeds, stream=None, torch_memory: bool = True) -> Net:
    if torch_memory:
        use_torch_allocator(True)
    n = len(params_list)
    arr = (DpsnnParams * n)(*[to_struct(p) for p in params_list])
    sd = (C.c_uint64 * n)(*[int(s) for s in seeds])
    h = C.c_void_p()
    _check("dpsnn_build_batch", lib().dpsnn_build_batch(arr, sd, n, C.byref(h)))
    net = Net(h, list(params_list), list(seeds))
    dpsnn_set_stream(net, current_torch_stream() if stream is None else stream)
    return net


def dpsnn_net_info(net: Net, k: int) -> dict:
    v = [C.c_int64(0) for _ in range(4)]
    _check("dpsnn_net_info", lib().dpsnn_net_info(net.h, int(k), *[C.byref(x) for x in v]))
    return {"base": v[0].value, "n_neurons": v[1].value, "module_base": v[2].value,
            "n_modules": v[3].value}


def dpsnn_set_stream(net: Net, stream) -> None:
    _check("dpsnn_set_stream", lib().dpsnn_set_stream(net.h, C.c_void_p(int(stream or 0))))


def dpsnn_step(net: Net, n_steps: int) -> None:
    _check("dpsnn_step", lib().dpsnn_step(net.h, int(n_steps)))


def dpsnn_set_schedule(net: Net, sched: int) -> None:
    _check("dpsnn_set_schedule", lib().dpsnn_set_schedule(net.h, int(sched)))


def dpsnn_set_delivery(net: Net, deliver_blocks: int = 0, spike_lists: int = -1) -> None:
    _check("dpsnn_set_delivery",
           lib().dpsnn_set_delivery(net.h, int(deliver_blocks), int(spike_lists)))


def dpsnn_set_routing(net: Net, route_blocks: int = 0) -> None:
    _check("dpsnn_set_routing", lib().dpsnn_set_routing(net.h, int(route_blocks)))


def dpsnn_set_graph_steps(net: Net, steps: int) -> None:
    _check("dpsnn_set_graph_steps", lib().dpsnn_set_graph_steps(net.h, int(steps)))


def dpsnn_autotune(net: Net, probe_steps: int) -> int:
    chosen = C.c_int32(-1)
    _check("dpsnn_autotune", lib().dpsnn_autotune(net.h, int(probe_steps), C.byref(chosen)))
    return int(chosen.value)


def dpsnn_profile_steps(net: Net, n_steps: int):
    """(update_ms, delivery_ms) summed over n_steps real steps."""
    ms = np.zeros(2, np.float64)
    _check("dpsnn_profile_steps", lib().dpsnn_profile_steps(net.h, int(n_steps), _ptr(ms)))
    return float(ms[0]), float(ms[1])


def dpsnn_sync(net: Net) -> int:
    return int(lib().dpsnn_sync(net.h))


def dpsnn_read_spikes(net: Net):
    n = C.c_int64(0)
    rc = lib().dpsnn_read_spikes(net.h, None, None, 0, C.byref(n))
    if rc not in (0, -5):
        _check("dpsnn_read_spikes", rc)
    st = np.zeros(n.value, np.int32)
    ids = np.zeros(n.value, np.int32)
    rc = lib().dpsnn_read_spikes(net.h, _ptr(st), _ptr(ids), n.value, C.byref(n))
    _check("dpsnn_read_spikes", rc)
    return st, ids


def dpsnn_read_log(net: Net):
    """(steps, ids) of the device spike log in device order (no drain)."""
    n = C.c_int64(0)
    _check("dpsnn_read_log", lib().dpsnn_read_log(net.h, None, None, 0, C.byref(n)))
    st = np.zeros(n.value, np.int32)
    ids = np.zeros(n.value, np.int32)
    _check("dpsnn_read_log",
           lib().dpsnn_read_log(net.h, _ptr(st), _ptr(ids), n.value, C.byref(n)))
    return st, ids


def dpsnn_read_spikes_net(net: Net, k: int):
    """(steps, network-local ids) of network k of a batch handle."""
    n = C.c_int64(0)
    rc = lib().dpsnn_read_spikes_net(net.h, int(k), None, None, 0, C.byref(n))
    if rc not in (0, -5):
        _check("dpsnn_read_spikes_net", rc)
    st = np.zeros(n.value, np.int32)
    ids = np.zeros(n.value, np.int32)
    rc = lib().dpsnn_read_spikes_net(net.h, int(k), _ptr(st), _ptr(ids), n.value, C.byref(n))
    _check("dpsnn_read_spikes_net", rc)
    return st, ids


def dpsnn_read_rates(net: Net) -> np.ndarray:
    nb = C.c_int64(0)
    _check("dpsnn_read_rates", lib().dpsnn_read_rates(net.h, None, 0, C.byref(nb)))
    out = np.zeros((max(nb.value, 0), net.M, net.n_pops), np.uint32)
    if nb.value > 0:
        _check("dpsnn_read_rates",
               lib().dpsnn_read_rates(net.h, _ptr(out), nb.value, C.byref(nb)))
    return out


def dpsnn_read_rates_net(net: Net, k: int) -> np.ndarray:
    """Rate bins [bins][modules of network k][n_pops] of network k."""
    nb = C.c_int64(0)
    _check("dpsnn_read_rates_net",
           lib().dpsnn_read_rates_net(net.h, int(k), None, 0, C.byref(nb)))
    m = dpsnn_net_info(net, k)["n_modules"]
    out = np.zeros((max(nb.value, 0), m, net.n_pops), np.uint32)
    if nb.value > 0:
        _check("dpsnn_read_rates_net",
               lib().dpsnn_read_rates_net(net.h, int(k), _ptr(out), nb.value, C.byref(nb)))
    return out


def dpsnn_stats(net: Net) -> dict:
    s = DpsnnStats()
    _check("dpsnn_stats", lib().dpsnn_stats(net.h, C.byref(s)))
    return {name: getattr(s, name) for name, _ in DpsnnStats._fields_}


dpsnn_stats_get = dpsnn_stats


def dpsnn_free(net: Net) -> None:
    net.close()


def dpsnn_strerror(code: int) -> str:
    return lib().dpsnn_strerror(int(code)).decode()


def dpsnn_read_state(net: Net):
    V = np.zeros(net.N, np.float32)
    c = np.zeros(net.N, np.float32)
    r = np.zeros(net.N, np.uint8)
    _check("dpsnn_read_state", lib().dpsnn_read_state(net.h, _ptr(V), _ptr(c), _ptr(r)))
    return V, c, r


def dpsnn_write_state(net: Net, V=None, c=None, ref=None) -> None:
    V = None if V is None else np.ascontiguousarray(V, np.float32)
    c = None if c is None else np.ascontiguousarray(c, np.float32)
    ref = None if ref is None else np.ascontiguousarray(ref, np.uint8)
    _check("dpsnn_write_state", lib().dpsnn_write_state(net.h, _ptr(V), _ptr(c), _ptr(ref)))


def dpsnn_read_slots(net: Net) -> np.ndarray:
    out = np.zeros((net.D, net.N), np.int64)
    _check("dpsnn_read_slots", lib().dpsnn_read_slots(net.h, _ptr(out)))
    return out


_W_NP = {W_F32: np.float32, W_F16: np.uint16, W_I8: np.int8}


def dpsnn_read_rows(net: Net, first: int, count: int):
    """(targets, stored efficacies, delay - d_min) of rows first..first+count-1,
    each row sorted by (target, delay, draw index)."""
    Ko = int(net.params["K_out"])
    wd = net.params["weight_dtype"]
    wd = WEIGHT_DTYPES[wd] if isinstance(wd, str) else int(wd)
    tgt = np.zeros((count, Ko), np.int32)
    w = np.zeros((count, Ko), _W_NP[wd])
    dk = np.zeros((count, Ko), np.uint8)
    _check("dpsnn_read_rows",
           lib().dpsnn_read_rows(net.h, int(first), int(count), _ptr(tgt), _ptr(w), _ptr(dk)))
    return tgt, w, dk


def dpsnn_read_plasticity(net: Net, first: int, count: int):
    """(last activation step, plasticity signal) of the synapses of rows
    first..first+count-1, in the order of dpsnn_read_rows."""
    Ko = int(net.params["K_out"])
    ta = np.zeros((count, Ko), np.int32)
    y = np.zeros((count, Ko), np.float32)
    _check("dpsnn_read_plasticity",
           lib().dpsnn_read_plasticity(net.h, int(first), int(count), _ptr(ta), _ptr(y)))
    return ta, y


def dpsnn_host_table(params: dict, name: str, dtype) -> np.ndarray:
    s = to_struct(params)
    nb = lib().dpsnn_host_table(C.byref(s), name.encode(), None, 0)
    if nb < 0:
        raise DpsnnError("dpsnn_host_table", int(nb))
    out = np.zeros(nb // np.dtype(dtype).itemsize, dtype)
    lib().dpsnn_host_table(C.byref(s), name.encode(), _ptr(out), nb)
    return out


# ---- slow-wave analysis (Sec. 2.3, Eq. 4) ---------------------------------
def _wave_params(net_index, n_bins, noise_var, seed, min_down, min_up, min_modules):
    return DpsnnWaveParams(ABI_VERSION, net_index, n_bins, noise_var, seed, min_down, min_up,
                           min_modules, 0)


def _wave_outputs(cap_tr, cap_w):
    return (np.zeros(cap_tr, np.int32), np.zeros(cap_tr, np.float64),
            np.zeros(cap_tr, np.int32), np.zeros(cap_w, np.float64),
            np.zeros(cap_w, np.float64), np.zeros(cap_w, np.int32))


def _wave_dict(res, o):
    nt, nw = int(res.n_transitions), int(res.n_waves)
    return {"bin0": int(res.bin0), "n_bins": int(res.n_bins), "n_transitions": nt,
            "n_waves": nw, "mean_speed": float(res.mean_speed), "module": o[0][:nt],
            "T": o[1][:nt], "wave": o[2][:nt], "speed": o[3][:nw], "t0": o[4][:nw],
            "n": o[5][:nw]}


def dpsnn_waves(net: Net, net_index: int = 0, n_bins: int = 0, noise_var: float = 0.5,
                seed: int = 1, min_down: int = 2, min_up: int = 2,
                min_modules: int = 1) -> dict:
    """Slow-wave analysis of the rate bins the handle holds (not drained)."""
    wp = _wave_params(net_index, n_bins, noise_var, seed, min_down, min_up, min_modules)
    res = DpsnnWaveResult()
    _check("dpsnn_waves", lib().dpsnn_waves(net.h, C.byref(wp), C.byref(res), None, None,
                                            None, 0, None, None, None, 0))
    o = _wave_outputs(int(res.n_transitions), int(res.n_waves))
    _check("dpsnn_waves", lib().dpsnn_waves(net.h, C.byref(wp), C.byref(res), _ptr(o[0]),
                                            _ptr(o[1]), _ptr(o[2]), len(o[0]), _ptr(o[3]),
                                            _ptr(o[4]), _ptr(o[5]), len(o[3])))
    return _wave_dict(res, o)


def _waves_counts(fn, counts, grid_w, grid_h, bin_steps, dt_ms, bin0, noise_var, seed,
                  min_down, min_up, min_modules):
    import torch
    assert counts.is_cuda and counts.is_contiguous() and counts.dim() == 3
    assert counts.dtype in (torch.int32, torch.uint32)
    nb, M, P = counts.shape
    wp = _wave_params(0, 0, noise_var, seed, min_down, min_up, min_modules)
    st = torch.cuda.current_stream().cuda_stream
    args = (C.c_void_p(counts.data_ptr()), nb, grid_w, grid_h, P, bin_steps, dt_ms, bin0,
            C.byref(wp), C.c_void_p(st))
    res = DpsnnWaveResult()
    f = getattr(lib(), fn)
    _check(fn, f(*args, C.byref(res), None, None, None, 0, None, None, None, 0))
    o = _wave_outputs(int(res.n_transitions), int(res.n_waves))
    _check(fn, f(*args, C.byref(res), _ptr(o[0]), _ptr(o[1]), _ptr(o[2]), len(o[0]),
                 _ptr(o[3]), _ptr(o[4]), _ptr(o[5]), len(o[3])))
    return _wave_dict(res, o)


def dpsnn_waves_counts(counts, grid_w: int, grid_h: int, bin_steps: int, dt_ms: float,
                       bin0: int = 0, noise_var: float = 0.5, seed: int = 1,
                       min_down: int = 2, min_up: int = 2, min_modules: int = 1) -> dict:
    """Slow-wave analysis of a device tensor of counts [bins][modules][pops]
    (uint32 data, e.g. a torch.int32 CUDA tensor)."""
    return _waves_counts("dpsnn_waves_counts", counts, grid_w, grid_h, bin_steps, dt_ms, bin0,
                         noise_var, seed, min_down, min_up, min_modules)


def dpsnn_waves_counts_static(counts, grid_w: int, grid_h: int, bin_steps: int,
                              dt_ms: float, bin0: int = 0, noise_var: float = 0.5,
                              seed: int = 1, min_down: int = 2, min_up: int = 2,
                              min_modules: int = 1) -> dict:
    """The same analysis with the library's fixed device scratch buffer: no
    device allocation (limits in include/dpsnn.h)."""
    return _waves_counts("dpsnn_waves_counts_static", counts, grid_w, grid_h, bin_steps,
                         dt_ms, bin0, noise_var, seed, min_down, min_up, min_modules)
