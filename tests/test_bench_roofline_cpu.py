"""The benchmark's sweep roofline on the CPU: the loop mixes the build
records from the kernels' assembly are priced with calibrated issue costs
and weighted by the wave steps the kernel counts; each texel encoding is
priced with its own kernel's loops (FP16 channels up to 11 bits, 16-bit
code values above).  Synthetic calibration figures stand in for the GPU's."""
import ctypes
import os

import pytest

import bench
from paper_1909_02294_amd import build as _b


@pytest.fixture(scope="module")
def calib():
    if not (os.path.exists(_b.MIX_JSON) and os.path.exists(_b.CALIB_LIB)):
        pytest.skip("library not built")
    lib = ctypes.CDLL(_b.CALIB_LIB)
    lib.ivde_calib_class_name.restype = ctypes.c_char_p
    names = [lib.ivde_calib_class_name(k).decode() for k in range(lib.ivde_calib_classes())]
    # every class the sweep prices exists in the library, in the index order bench.py assumes
    assert max(k for _, k in bench._CLASS_OF) < len(names)
    assert names[18] == "v_cvt_f32_u32_sdwa" and names[7] == "v_fma_mix_f32"
    half = {"v_fma_mix_f32", "v_med3_f32", "v_fract_f32", "v_cvt_i32_f32", "v_cvt_f32_u32_sdwa", "v_cmp_f32",
            "v_cndmask_b32", "v_mad_u32_u24", "v_lshlrev_b32", "v_addc_co_u32"}
    valu = {n: {"cycles": 8.0 if n == "v_rcp_f32" else 4.0 if n in half else 2.0, "clock_ghz": 2.3} for n in names}
    return {"valu": valu, "gather": {"cycles_per_load_per_cu": 16.0, "clock_ghz": 2.3}}


@pytest.mark.parametrize("px", [2, 4])
def test_each_encoding_priced_with_its_own_loops(calib, px):
    evals, sweep_s = 2.97e10, 0.03
    steps = (evals / 64, evals / 64, 0.8 * evals / 64)     # every step on projected records, 80% inside the band
    out = {}
    for bits in (10, 12, 16):
        r, loops = bench.sweep_roofline(evals, sweep_s, calib, None, px, steps, bits)
        pre = ("pairs" if px == 2 else "quads") + ("16" if bits > 11 else "")
        assert set(loops) == {pre + "_inside", pre + "_tested", pre + "_records"}
        assert sum(r["wave_steps"].values()) == pytest.approx(evals / 64)
        assert ("16-bit code values" in r["kernel"]) == (bits > 11)
        assert r["traffic"] is None
        for unit in ("valu", "gather"):
            assert r[unit]["frac"] == pytest.approx(r[unit]["achieved"] / r[unit]["peak"])
        assert r["frac"] == max(r["valu"]["frac"], r["gather"]["frac"])
        out[bits] = r
    # the same gathers at every depth; the 16-bit channels' decode costs issue slots
    assert out[12]["gather"] == out[10]["gather"]
    assert out[12]["valu"]["valu_instructions_per_wave_step"] > out[10]["valu"]["valu_instructions_per_wave_step"]
    assert out[16]["valu"] == out[12]["valu"]
    conv = loops_for(calib, px, 12)
    assert conv.get("v_cvt_f32_u32_sdwa", {}).get("class") == "v_cvt_f32_u32_sdwa"


def loops_for(calib, px, bits):
    evals = 2.97e10
    _, loops = bench.sweep_roofline(evals, 0.03, calib, None, px, (evals / 64, evals / 64, evals / 64), bits)
    return loops[("pairs" if px == 2 else "quads") + ("16" if bits > 11 else "") + "_inside"]
