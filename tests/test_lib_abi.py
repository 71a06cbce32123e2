"""CPU checks of the C ABI: the built library exports every function that
include/ilt.h declares, and the Python binding's struct layouts match the C
header (sizes and offsets from a gcc-compiled probe).  No GPU work."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ilt.h")
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
                 if f.endswith(".h"))


def _declared_functions():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"^\s*(?:const\s+)?(?:long\s+long|unsigned\s+\w+|\w+)\s*\*?\s*(\w+)\s*\(", src,
                                flags=re.M))
    return sorted(names)


def test_header_declares_the_five_calls():
    names = _declared_functions()
    for n in ("litho_forward", "litho_adjoint", "levelset_step", "edt_reinit", "ilt_solve",
              "ilt_create", "ilt_destroy", "ilt_last_error", "resist_loss", "ilt_solve_batch", "ilt_autotune",
              "dsn_create", "dsn_forward", "dsn_backward", "dsn_adam_step", "dsn_predict", "dsn_num_params"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2303_12529_amd import ilt
    if not os.path.exists(ilt.LIB_PATH):
        pytest.skip("libilt.so not built")
    lib = ctypes.CDLL(ilt.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layouts_match_header():
    from paper_2303_12529_amd import ilt
    probe = r'''
#include <stdio.h>
#include <stddef.h>
#include "ilt.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(ilt_optics), sizeof(ilt_corner), sizeof(ilt_params), sizeof(ilt_report));
  printf("%zu %zu %zu\n", offsetof(ilt_params, eta), offsetof(ilt_params, n_corners), offsetof(ilt_params, corners));
  printf("%zu %zu\n", offsetof(ilt_optics, h_kernels), offsetof(ilt_report, loss));
  printf("%zu %zu %zu %d %d %d\n", sizeof(ilt_clip), offsetof(ilt_clip, d_trace), offsetof(ilt_clip, params),
         ILT_BATCH_MAX_SIZES, ILT_BATCH_MAX_LANES, ILT_BATCH_MAX_CLIPS);
  printf("%zu %zu %zu\n", sizeof(ilt_tuning), offsetof(ilt_tuning, xcd_remap), offsetof(ilt_tuning, st_xsplit));
  printf("%zu %zu\n", offsetof(ilt_params, optimizer), offsetof(ilt_params, iter0));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "p.c")
        exe = os.path.join(d, "p")
        open(c, "w").write(probe)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, c])
        out = subprocess.check_output([exe]).decode().split()
    vals = [int(v) for v in out]
    assert vals[0] == ctypes.sizeof(ilt._Optics)
    assert vals[1] == ctypes.sizeof(ilt._Corner)
    assert vals[2] == ctypes.sizeof(ilt._Params)
    assert vals[3] == ctypes.sizeof(ilt._Report)
    assert vals[4] == ilt._Params.eta.offset
    assert vals[5] == ilt._Params.n_corners.offset
    assert vals[6] == ilt._Params.corners.offset
    assert vals[7] == ilt._Optics.h_kernels.offset
    assert vals[8] == ilt._Report.loss.offset
    assert vals[9] == ctypes.sizeof(ilt._Clip)
    assert vals[10] == ilt._Clip.d_trace.offset
    assert vals[11] == ilt._Clip.params.offset
    assert tuple(vals[12:15]) == (ilt.ILT_BATCH_MAX_SIZES, ilt.ILT_BATCH_MAX_LANES, ilt.ILT_BATCH_MAX_CLIPS)
    assert vals[15] == ctypes.sizeof(ilt._Tuning) and vals[16] == ilt._Tuning.xcd_remap.offset
    assert vals[17] == ilt._Tuning.st_xsplit.offset
    assert vals[18] == ilt._Params.optimizer.offset
    assert vals[19] == ilt._Params.iter0.offset


def test_params_roundtrip_and_validation():
    from paper_2303_12529_amd import ilt
    from paper_2303_12529_amd.inputs import WORKLOADS
    p = ilt.Params.from_dict(WORKLOADS["c1"]["params"])
    c = p.to_c()
    assert c.n_corners == 3 and c.corners[2].set == 1
    assert abs(c.corners[1].dose - 1.02) < 1e-6 and abs(c.corners[2].omega - 7.5) < 1e-6
    assert c.d_lower == -100.0 and c.d_upper == 900.0
    with pytest.raises(ValueError):
        ilt.Params(corners=()).to_c()


def test_bench_refuses_multi_gpu():
    r = subprocess.run(["python", os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr
