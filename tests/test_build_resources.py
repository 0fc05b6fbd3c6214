"""Register budget of the built kernels, from the resource usage the compiler reports
at build time (kept beside the objects by the build).

* No kernel spills vector registers or uses scratch memory. A spill is private memory
  traffic the byte model does not count (scalar registers spill into vector-register
  lanes, not memory, and are allowed): two spilled values of the fused FP32 first launch at p = 3
  once cost 7 MB per launch of extra HBM traffic, the whole gap between the counted and
  the algorithmic bytes.
* The fused FP32 stage kernels keep the occupancy their LDS sizing is made for: at
  least 4 waves per SIMD for the first launch and 5 for the second at 3D p = 3, and the
  first launch's LDS lets 4 workgroups share one compute unit's 160 KB.
"""
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "_build")


def resources(src):
    path = os.path.join(BUILD, src + ".resources.json")
    if not os.path.exists(path):
        pytest.skip(f"{src} not built with resource reporting")
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("src", ["fr_kernels.hip", "fr_fwh.hip"])
def test_no_kernel_spills(src):
    r = resources(src)
    assert r, src
    spilled = {k: v for k, v in r.items() if v.get("vgpr_spill", 0) or v.get("scratch", 0)}
    assert not spilled, spilled


def test_fused_fp32_stage_kernels_keep_their_occupancy():
    r = resources("fr_kernels.hip")
    a = r["_ZN2fr9k_stage_aIfLi3ELi3ELb0EEEvNS_5KArgsIT_EEPKS2_i"]
    assert a["occupancy"] >= 4 and 4 * a["lds"] <= 160 * 1024, a
    for mode in range(4):
        b = r[f"_ZN2fr9k_stage_bIfLi3ELi3ELi{mode}ELb0EEEvNS_5KArgsIT_EE"]
        assert b["occupancy"] >= 5 and 5 * b["lds"] <= 160 * 1024, b
