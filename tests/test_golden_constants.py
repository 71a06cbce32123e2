"""The constants the paper states (tests/golden/paper_constants.json, each
with its citation) against the workload definitions, the C-ABI headers and
the oracle.  The curvature weight lambda is not among them: the workloads take
their configuration's value, 0.05, instead of the paper's 0.9."""
import json
import os
import re

import pytest

from oracle import dsn as o_dsn
from paper_2303_12529_amd import develset
from paper_2303_12529_amd.inputs import workload_inputs

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def paper():
    with open(os.path.join(HERE, "golden", "paper_constants.json")) as f:
        d = json.load(f)
    for k, v in d.items():
        if not k.startswith("_"):
            assert v["cite"].startswith("Sec. "), k
    return {k: v["value"] for k, v in d.items() if not k.startswith("_")}


@pytest.mark.parametrize("workload,pixel_nm", [("c0", 8.0), ("c1", 1.0)])
def test_tsdf_bounds_and_resist_steepness(paper, workload, pixel_nm):
    _, _, _, prm = workload_inputs(workload, 0)
    # the bounds are stated in nm; phi is stored in pixels
    assert prm["d_upper"] * pixel_nm == paper["D_u_nm"]
    assert prm["d_lower"] * pixel_nm == paper["D_l_nm"]
    assert prm["sigma_z"] == paper["sigma_z"]
    assert prm["eta"] == paper["eta"]


def test_kernels_and_corner_weights(paper):
    _, H, w, prm = workload_inputs("c1", 0)
    assert H.shape[1] == paper["N_h"]
    weights = [c[2] for c in prm["corners"]]
    assert weights[0] == paper["alpha"]
    assert all(x == paper["beta"] for x in weights[1:]) and len(weights) == 3


def test_heaviside_width(paper):
    from paper_2303_12529_amd import dsn
    assert dsn.EPS_AHF == paper["epsilon"]
    assert o_dsn.EPS_AHF == paper["epsilon"]
    with open(os.path.join(ROOT, "include", "dsn.h")) as f:
        m = re.search(r"#define\s+DSN_EPS_AHF\s+([0-9.eE+-]+)f?", f.read())
    assert m and float(m.group(1)) == paper["epsilon"]


def test_modulation_shift_range(paper):
    lo, hi = paper["delta_h_range"]
    assert min(develset.MOD_SHIFTS) == lo and max(develset.MOD_SHIFTS) == hi
