"""The ctypes structures of the Python binding match the C layout of
include/dngd.h (sizes and field offsets, from a C program built here)."""
import ctypes as C
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROG = r"""
#include <stdio.h>
#include <stddef.h>
#include "dngd.h"
#define P(T, F) printf(#T " " #F " %zu\n", offsetof(T, F));
int main(void) {
  printf("dngd_step_opts size %zu\n", sizeof(dngd_step_opts));
  printf("dngd_step_stats size %zu\n", sizeof(dngd_step_stats));
  printf("dngd_iter_stats size %zu\n", sizeof(dngd_iter_stats));
  printf("dngd_problem_desc size %zu\n", sizeof(dngd_problem_desc));
  printf("dngd_refine size %zu\n", sizeof(dngd_refine));
  P(dngd_step_opts, eps_norm) P(dngd_step_opts, landmarks) P(dngd_step_opts, ir_tol)
  P(dngd_step_opts, fvv_out) P(dngd_step_opts, nystrom_chunk_rows) P(dngd_step_opts, nystrom_reuse)
  P(dngd_step_opts, pcg_kvp)
  P(dngd_step_stats, ga_accepted) P(dngd_step_stats, ir_residual)
  P(dngd_step_stats, ms_gram_kernel) P(dngd_step_stats, gram_attempts)
  P(dngd_step_stats, nystrom_shift) P(dngd_step_stats, nystrom_reused)
  P(dngd_step_stats, pcg_escalated) P(dngd_step_stats, gram_start_passes)
  P(dngd_iter_stats, eta_index) P(dngd_iter_stats, step)
  P(dngd_problem_desc, kappa) P(dngd_problem_desc, x_int) P(dngd_problem_desc, g_init)
  P(dngd_refine, n) P(dngd_refine, j_dtype) P(dngd_refine, sweeps) P(dngd_refine, lambda)
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_struct_layout_matches_header():
    from paper_2505_21404_amd import dngd as D
    with tempfile.TemporaryDirectory() as tmp:
        src = os.path.join(tmp, "layout.c")
        exe = os.path.join(tmp, "layout")
        with open(src, "w") as f:
            f.write(PROG)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), src, "-o", exe],
                       check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        t, f, v = line.split()
        got[(t, f)] = int(v)
    py = {"dngd_step_opts": D.StepOpts, "dngd_step_stats": D.StepStats,
          "dngd_iter_stats": D.IterStats, "dngd_problem_desc": D.ProblemDesc,
          "dngd_refine": D.Refine}
    rename = {"lambda": "lam"}
    for (t, f), v in got.items():
        cls = py[t]
        if f == "size":
            assert C.sizeof(cls) == v, (t, C.sizeof(cls), v)
        else:
            assert getattr(cls, rename.get(f, f)).offset == v, (t, f)
