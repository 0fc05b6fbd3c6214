"""Register budget of the built kernels, from the resource usage the compiler reports
at build time (kept beside the objects by the build).

* No kernel spills vector registers or uses scratch memory. A spill is private memory
  traffic the byte model does not count (scalar registers spill into vector-register
  lanes, not memory, and are allowed): two spilled values of the fused FP32 first launch at p = 3
  once cost 7 MB per launch of extra HBM traffic, the whole gap between the counted and
  the algorithmic bytes.
* The fused FP32 stage kernels keep the occupancy their LDS sizing is made for at 3D
  p = 3: the first launch with stored metrics at least 4 waves per SIMD, with metrics
  formed from the geometry nodes at least 3 (its FP64 metric products need the larger
  register budget), its LDS letting that many workgroups share one compute unit's
  160 KB; the second launch at least 5 waves in both variants.
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
    # template arguments after the order: metric source (0 from the nodes, 1 stored, 2
    # mortar groups, 3 extruded columns), the tile shape (0 default, 1 half the elements,
    # 2 a quarter, 3 matrix cores), and the neighbour exchange (0 gather, 1 scatter)
    for fv, waves in ((0, 3), (1, 4), (3, 4)):
        for tile in range(4):
            for scat in (0, 1):
                a = r[f"_ZN2fr9k_stage_aIfLi3ELi3ELi{fv}ELi{tile}ELb{scat}EEEvNS_5KArgsIT_EEPKS2_i"]
                assert a["occupancy"] >= waves and waves * a["lds"] <= 160 * 1024, (fv, tile, scat, a)
    for fv in (0, 1):
        for tile in range(3):
            for scat in (0, 1):
                for mode in range(4):
                    b = r[f"_ZN2fr9k_stage_bIfLi3ELi3ELi{mode}ELi{fv}ELi{tile}ELb{scat}EEEvNS_5KArgsIT_EE"]
                    assert b["occupancy"] >= 5 and 5 * b["lds"] <= 160 * 1024, (fv, tile, scat, mode, b)
