"""The Python binding's ctypes structures match include/mc.h: a C program
compiled here with gcc against the header prints sizeof and offsetof of
every field the binding declares, and both must agree (a field added to
the header but not to the binding, or in another order, fails here rather
than on the GPU)."""
import os
import shutil
import subprocess

import pytest

from paper_2501_06910_amd import mc as M

HERE = os.path.dirname(os.path.abspath(__file__))
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
ROCM_INCLUDE = "/opt/rocm/include"

PAIRS = {
    "mc_grid": M.McGrid, "mc_plan_opts": M.McPlanOpts, "mc_plan_info": M.McPlanInfo, "mc_params": M.McParams,
    "mc_result": M.McResult, "mc_codes": M.McCodes, "mc_train_opts": M.McTrainOpts,
    "mc_batch_item": M.McBatchItem, "mc_tuning": M.McTuning, "mc_batch_ditem": M.McBatchDItem,
}


@pytest.mark.skipif(shutil.which("gcc") is None or not os.path.isdir(ROCM_INCLUDE), reason="gcc or ROCm headers")
def test_ctypes_layout_matches_header(tmp_path):
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "mc.h"', 'int main(void) {']
    expect = []
    for cname, cls in PAIRS.items():
        lines.append(f'    printf("%zu\\n", sizeof({cname}));')
        expect.append((cname, "sizeof", C_sizeof(cls)))
        for fname, _ in cls._fields_:
            lines.append(f'    printf("%zu\\n", offsetof({cname}, {fname}));')
            expect.append((cname, fname, getattr(cls, fname).offset))
    lines += ['    return 0;', '}']
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "abi"
    r = subprocess.run(["gcc", "-std=c11", "-D__HIP_PLATFORM_AMD__", f"-I{INCLUDE}", f"-I{ROCM_INCLUDE}", str(src),
                        "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert len(got) == len(expect)
    bad = [(c, f, e, g) for (c, f, e), g in zip(expect, got) if e != g]
    assert not bad, bad


def C_sizeof(cls):
    import ctypes
    return ctypes.sizeof(cls)
