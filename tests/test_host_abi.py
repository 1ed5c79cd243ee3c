"""Host-side checks of libdpsnn that need no GPU: the shared library loads
and exports every entry point include/dpsnn.h declares, its host tables are
bitwise equal to the oracle's (computed independently from the same
definitions), and invalid parameter sets are rejected."""
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1902_08410_amd import dpsnn as L
from paper_1902_08410_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dpsnn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dpsnn_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_entry_point():
    lib = L.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.EXPORTS) == names


def test_strerror_names_codes():
    assert L.dpsnn_strerror(0) == "ok"
    assert "spike log" in L.dpsnn_strerror(-5)
    assert L.dpsnn_strerror(-99) == "unknown error"


TABLES = [("prop_f64", np.float64), ("prop_f32", np.float32), ("n_arp", np.int32),
          ("pois_thr_0", np.uint32), ("pois_thr_1", np.uint32), ("off_thr", np.uint32),
          ("off_xy", np.int32), ("s8", np.float32), ("s8fix", np.int64)]
for _q in (0, 1):
    TABLES += [(f"wt64_{_q}", np.float64), (f"wt32_{_q}", np.float32),
               (f"wt16_{_q}", np.uint16), (f"wq8_{_q}", np.int8), (f"wfix_{_q}", np.int64),
               (f"jx64_{_q}", np.float64), (f"jx32_{_q}", np.float32),
               (f"jxfix_{_q}", np.int64)]

PARAM_SETS = {
    "2x2_swa": W.swa(),
    "24x24_aw": W.grid(24, 24, "aw"),
    "48x48_f16_l05": W.grid(48, 48, "swa", **{"lambda": 0.5, "weight_dtype": "f16"}),
    "48x48_i8_l4": W.grid(48, 48, "aw", **{"lambda": 4.0, "weight_dtype": "i8"}),
    "96x96_i8_q32": W.grid(96, 96, "swa", **{"lambda": 2.0, "weight_dtype": "i8",
                                          "acc_bits": 64, "q_frac_bits": 32}),
    "tiny_3x2": W.tiny(w=3, h=2, K=16, K_out=8, tau_c=[300.0, 300.0], I_const=[0.5, 0.2]),
    "odd_7x5": W.grid(7, 5, "swa", **{"lambda": 1.7, "J_sd": [0.3, 0.9]}),
    "open_6x3": W.grid(6, 3, "aw", torus=0, **{"lambda": 1.3}),
}


@pytest.mark.parametrize("name", sorted(PARAM_SETS))
def test_host_tables_bitwise_equal_to_oracle(name):
    p = PARAM_SETS[name]
    o = O.Oracle(p, 1, store_rows=False) if p["grid_w"] * p["grid_h"] <= 64 else None
    if o is None:
        # tables do not depend on the network size beyond the grid: build the
        # oracle's tables on a network with the same grid and K = 4
        o = O.Oracle(dict(p, K=5, K_out=4, frac_local=[0.5, 0.5]), 1, store_rows=False)
    for tname, dt in TABLES:
        a = L.dpsnn_host_table(p, tname, dt)
        b = o.table(tname, dt)
        if tname.startswith(("wfix", "jxfix")) and p["acc_bits"] == 32:
            assert np.all(np.abs(a) < 2**31)
        assert a.dtype == b.dtype and a.shape == b.shape, tname
        assert a.tobytes() == b.tobytes(), (name, tname)


def test_f16_table_matches_numpy_rounding():
    p = W.grid(4, 4, "swa", weight_dtype="f16", J_sd=[0.7, 1.3])
    for q in (0, 1):
        w64 = L.dpsnn_host_table(p, f"wt64_{q}", np.float64)
        h = L.dpsnn_host_table(p, f"wt16_{q}", np.uint16)
        assert np.array_equal(h, w64.astype(np.float16).view(np.uint16))


@pytest.mark.parametrize("bad", [
    dict(torus=2), dict(d_min=0), dict(d_max=0), dict(d_min=1, d_max=65),
    {"lambda": 0.0}, {"lambda": -1.0}, dict(grid_w=1, grid_h=1), dict(K=3),
    dict(K_out=5000), dict(acc_bits=16), dict(q_frac_bits=31), dict(weight_dtype=3),
    dict(rate_bin_steps=0), dict(rate_bins_cap=0), dict(spike_log_cap=-1),
    dict(dt_ms=0.0), dict(tau_m=[0.0, 10.0]), dict(frac_exc=1.5),
    dict(frac_local=[1.2, 0.5]), dict(tau_arp=[30.0, 1.0]),
    dict(grid_w=64, grid_h=64, K=20000, K_out=10),   # more than 2^26 neurons
    # plasticity: binary32 efficacies only, positive constants
    dict(plastic=2),
    dict(plastic=1, weight_dtype="f16", stdp_update_steps=100, stdp_tau_plus=2.0,
         stdp_tau_minus=2.0, stdp_tau_y=5.0, stdp_w_max=1.0),
    dict(plastic=1, stdp_update_steps=0, stdp_tau_plus=2.0, stdp_tau_minus=2.0,
         stdp_tau_y=5.0, stdp_w_max=1.0),
    dict(plastic=1, stdp_update_steps=100, stdp_tau_plus=0.0, stdp_tau_minus=2.0,
         stdp_tau_y=5.0, stdp_w_max=1.0),
    dict(plastic=1, stdp_update_steps=100, stdp_tau_plus=2.0, stdp_tau_minus=2.0,
         stdp_tau_y=5.0, stdp_w_max=0.0),
    dict(plastic=1, stdp_update_steps=100, stdp_A_minus=-1.0, stdp_tau_plus=2.0,
         stdp_tau_minus=2.0, stdp_tau_y=5.0, stdp_w_max=1.0),
])
def test_invalid_parameters_rejected(bad):
    p = W.swa(rate_bins_cap=16, spike_log_cap=16)
    p.update(bad)
    with pytest.raises(L.DpsnnError) as e:
        L.dpsnn_host_table(p, "prop_f64", np.float64)
    assert e.value.code == -1


def test_single_module_valid_when_all_local():
    p = W.swa(grid_w=1, grid_h=1, frac_local=[1.0, 1.0])
    assert len(L.dpsnn_host_table(p, "prop_f64", np.float64)) == 8
    assert len(L.dpsnn_host_table(p, "off_xy", np.int32)) == 0


def test_abi_version_checked():
    s = L.to_struct(W.swa())
    s.abi_version = 99
    import ctypes as C
    assert L.lib().dpsnn_host_table(C.byref(s), b"prop_f64", None, 0) == -1


def test_struct_layout_matches_header(tmp_path):
    """Sizes and field offsets of the ctypes structs equal those of the C
    header (compiled here with the host C compiler)."""
    import ctypes as C
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    lines = []
    for cname, py in (("dpsnn_params", L.DpsnnParams), ("dpsnn_stats_t", L.DpsnnStats)):
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            cf = "lambda" if f == "lambda_" else f
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {cf}));')
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"dpsnn.h\"\n"
                   "int main(void) {\n" + "\n".join(lines) + "\nreturn 0; }\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(root, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for ln in out.splitlines():
        a, b, v = ln.split()
        got[(a, b)] = int(v)
    for cname, py in (("dpsnn_params", L.DpsnnParams), ("dpsnn_stats_t", L.DpsnnStats)):
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_queue_cap_validated():
    for cap in (-2, (1 << 20) + 1):
        with pytest.raises(L.DpsnnError) as e:
            L.dpsnn_host_table(W.swa(queue_cap=cap), "prop_f64", np.float64)
        assert e.value.code == -1
    for cap in (-1, 0, 1, 1 << 20):
        assert len(L.dpsnn_host_table(W.swa(queue_cap=cap), "prop_f64", np.float64)) == 8


# population model (Sec. 2.2, Table S1): F/B/I populations, per-pair
# efficacies, Eq. 1 from d = 0, open or periodic boundaries
POP_SETS = {
    "fbi_sw_open_6x5": W.fbi(6, 5, "sw", scale=0.05),
    "fbi_aw88_torus_4x4_f16": W.fbi(4, 4, "aw88", scale=0.05, open_boundary=0,
                                   weight_dtype="f16", lam=0.7),
    "fbi_aw28_open_i8_q32": W.fbi(5, 3, "aw28", scale=0.05, weight_dtype="i8",
                                 acc_bits=64, q_frac_bits=32, lam=0.4),
}


@pytest.mark.parametrize("name", sorted(POP_SETS))
def test_population_model_tables_bitwise_equal_to_oracle(name):
    p = POP_SETS[name]
    o = O.Oracle(p, 1, store_rows=False)
    names = [("prop_f64", np.float64), ("prop_f32", np.float32), ("n_arp", np.int32),
             ("off_thr", np.uint32), ("off_xy", np.int32), ("s8", np.float32),
             ("s8fix", np.int64), ("blocks", np.int32)]
    for q in range(3):
        names += [(f"pois_thr_{q}", np.uint32), (f"jx64_{q}", np.float64),
                  (f"jx32_{q}", np.float32), (f"jxfix_{q}", np.int64)]
        for b in range(3):
            names += [(f"wt64_{q}_{b}", np.float64), (f"wt32_{q}_{b}", np.float32),
                      (f"wt16_{q}_{b}", np.uint16), (f"wq8_{q}_{b}", np.int8),
                      (f"wfix_{q}_{b}", np.int64)]
    for tname, dt in names:
        a = L.dpsnn_host_table(p, tname, dt)
        b = o.table(tname, dt)
        assert a.dtype == b.dtype and a.shape == b.shape, (name, tname)
        assert a.tobytes() == b.tobytes(), (name, tname)
    blocks = L.dpsnn_host_table(p, "blocks", np.int32).reshape(3, 4, 4)
    # blocks of source s: (0.9 K_t synapses, population t's range, rule)
    lo = np.cumsum([0] + p["pop_size"][:2])
    for s in range(3):
        for t in range(3):
            n, a, b, rule = blocks[s, t]
            assert n == p["n_syn"][t][s] and a == lo[t] and b == lo[t] + p["pop_size"][t]
            assert rule == (2 if p["pop_exc"][s] else 0)


def test_population_model_invalid_parameters_rejected():
    base = W.fbi(3, 3, "sw", scale=0.05)
    bad = [dict(pop_size=[5, 38, 13]),                       # does not sum to K
           dict(n_syn=[[11, 11, 11], [34, 34, 34], [11, 11, 12]]),  # unequal rows
           dict(n_pops=5), dict(open_boundary=2)]
    for over in bad:
        with pytest.raises(L.DpsnnError) as e:
            L.dpsnn_host_table(dict(base, **over), "prop_f64", np.float64)
        assert e.value.code == -1, over


def test_wave_analysis_rejects_invalid_requests_before_any_device_call():
    """Argument checks of dpsnn_waves_counts / dpsnn_waves come first: none of
    these calls touches the device (the count pointer is never read)."""
    import ctypes as C
    lib = L.lib()
    fake = C.c_void_p(0x1000)
    res = L.DpsnnWaveResult()

    def call(nb=10, w=4, h=4, pops=2, bin_steps=50, dt=0.1, bin0=0, **kw):
        f = dict(abi_version=L.ABI_VERSION, net=0, n_bins=0, noise_var=0.5, seed=1,
                 min_down=2, min_up=2, min_modules=1, reserved=0)
        f.update(kw)
        wp = L.DpsnnWaveParams(**f)
        return lib.dpsnn_waves_counts(fake, nb, w, h, pops, bin_steps, dt, bin0, C.byref(wp),
                                      None, C.byref(res), None, None, None, 0, None, None,
                                      None, 0)

    E = -1  # DPSNN_E_INVAL
    assert call(nb=4097) == E            # more than 4096 bins
    assert call(nb=0) == E
    assert call(w=128, h=65) == E        # more than 8192 modules
    assert call(w=0) == E
    assert call(pops=0) == E
    assert call(bin_steps=0) == E
    assert call(dt=0.0) == E
    assert call(bin0=-1) == E
    assert call(min_down=0) == E
    assert call(min_up=0) == E
    assert call(min_modules=-1) == E
    assert call(noise_var=-0.5) == E
    assert call(noise_var=float("inf")) == E
    assert call(abi_version=1) == E
    wp = L.DpsnnWaveParams(L.ABI_VERSION, 0, 0, 0.5, 1, 2, 2, 1, 0)
    assert lib.dpsnn_waves(None, C.byref(wp), C.byref(res), None, None, None, 0, None, None,
                           None, 0) == E


def test_handle_setters_reject_a_null_handle():
    """The setters check their handle before touching the device."""
    from paper_1902_08410_amd import dpsnn as L
    lib = L.lib()
    E = -1
    assert lib.dpsnn_set_delivery(None, 0, -1) == E
    assert lib.dpsnn_set_delivery(None, 256, 1) == E
    assert lib.dpsnn_set_schedule(None, L.SCHED_SPLIT) == E
    assert lib.dpsnn_set_graph_steps(None, 64) == E


@pytest.mark.parametrize("over", [
    # the external sum of one step leaves int32 at Q = 16
    dict(Jext_mean=[20000.0, 20000.0], Jext_sd=[0.0, 0.0], nu_ext_hz=[30000.0, 30000.0]),
    # a single efficacy does not fit int32 at Q = 16
    dict(J_mean=[40000.0, -2.0]),
    # a plastic efficacy may grow to w_max = 2^15 mV = 2^31 at Q = 16
    dict(plastic=1, stdp_update_steps=100, stdp_tau_plus=2.0, stdp_tau_minus=2.0,
         stdp_tau_y=5.0, stdp_w_max=32768.0),
])
def test_fixed_point_range_errors_before_any_device_call(over):
    """DPSNN_E_RANGE: the int32 bounds that the parameters alone decide are
    checked on the host (tables and dpsnn_build) before any device work; the
    same parameters with int64 slots (Q = 32) are valid."""
    import ctypes as C
    p = W.swa(rate_bins_cap=16, spike_log_cap=16, **over)
    with pytest.raises(L.DpsnnError) as e:
        L.dpsnn_host_table(p, "prop_f64", np.float64)
    assert e.value.code == -4
    h = C.c_void_p()
    assert L.lib().dpsnn_build(C.byref(L.to_struct(p)), C.c_uint64(1), C.byref(h)) == -4
    assert not h.value
    if not over.get("plastic"):
        p64 = dict(p, acc_bits=64, q_frac_bits=32)
        assert len(L.dpsnn_host_table(p64, "prop_f64", np.float64)) == 8


def test_static_wave_scratch_rejects_oversized_requests_before_any_device_call():
    """dpsnn_waves_counts_static checks that the request fits its fixed
    64 MiB device buffer before touching the device: 90x90 modules and 4096
    bins need about 600 MB (the counts pointer is never dereferenced)."""
    import ctypes as C
    lib = L.lib()
    wp = L.DpsnnWaveParams(L.ABI_VERSION, 0, 0, 0.5, 1, 2, 2, 1, 0)
    res = L.DpsnnWaveResult()
    fake = C.c_void_p(0x1000)
    rc = lib.dpsnn_waves_counts_static(fake, 4096, 90, 90, 2, 50, 0.1, 0, C.byref(wp), None,
                                       C.byref(res), None, None, None, 0, None, None, None, 0)
    assert rc == -8
    assert "scratch" in L.dpsnn_strerror(-8)
    bad = L.DpsnnWaveParams(L.ABI_VERSION, 0, 0, 0.5, 1, 0, 2, 1, 0)   # min_down 0
    rc = lib.dpsnn_waves_counts_static(fake, 10, 3, 3, 2, 50, 0.1, 0, C.byref(bad), None,
                                       C.byref(res), None, None, None, 0, None, None, None, 0)
    assert rc == -1
