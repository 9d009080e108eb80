"""The oracle's pins must catch plausible mistakes (CPU only).

Each case plants one mistake into a copy of ``oracle/bfvm_oracle.c``, builds
it into a temporary library and runs the pin suites against it in a child
process; the pins must fail.  Nothing here touches the GPU path.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "bfvm_oracle.c")
PINS = ["tests/test_oracle_dense.py", "tests/test_oracle_invariants.py", "tests/test_oracle_adjoint.py"]

MUTANTS = {
    "end_diagonal_2r": ("b = 1.0 + r + beta;", "b = 1.0 + 2.0 * r + beta;"),
    "decay_not_split": ("double beta = dt * lambda[s] / 3.0;", "double beta = dt * lambda[s];"),
    "literal_plus_a": ("double a = -r;", "double a = r;"),
    "forward_axpy_sign": ("+ r[s] * base[(i - 1) * inner + j])", "- r[s] * base[(i - 1) * inner + j])"),
    "back_sub_index": ("cprime[s * n + i] * base[(i + 1) * inner + j]", "cprime[s * n + i + 1] * base[(i + 1) * inner + j]"),
    "y_view_transposed": ("*outer = nz; *n = ny; *inner = nx * S;", "*outer = nz; *n = nx; *inner = ny * S;"),
    "spacing_of_x_everywhere": ("r[s] = dt * D[s] / (h[axis] * h[axis]);", "r[s] = dt * D[s] / (h[0] * h[0]);"),
    "source_q_without_secretion": ("(*Q)[m * S + s] += secretion[k * S + s] + uptake[k * S + s];", "(*Q)[m * S + s] += uptake[k * S + s];"),
    "source_p_without_dt": ("(*P)[i * S + s] = dt * (*P)[i * S + s];", "(*P)[i * S + s] = (*P)[i * S + s];"),
    "dirichlet_once_per_step": ("            oracle_dirichlet(u, nsub, ndir, dir_voxel, dir_value, dir_active);   /* Dir */", "            if (a == 0) oracle_dirichlet(u, nsub, ndir, dir_voxel, dir_value, dir_active);"),
    "adjoint_transposed_index": ("g[i * inner] - cprime[i - 1] * g[(i - 1) * inner]", "g[i * inner] - cprime[i] * g[(i - 1) * inner]"),
    "adjoint_beta_sign": ("Gb[s] -= yx;", "Gb[s] += yx;"),
    "adjoint_laplacian_end": ("else if (i == n - 1) Lx = xl[i * inner] - xl[(i - 1) * inner];", "else if (i == n - 1) Lx = 2.0 * xl[i * inner] - xl[(i - 1) * inner];"),
    "adjoint_no_source_transpose": ("g[mvox[i] * S + s] = g[mvox[i] * S + s] / Q[i * S + s];", "g[mvox[i] * S + s] = g[mvox[i] * S + s];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor must match exactly once"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c99", "-shared", "-fPIC",
                    "-o", str(lib), str(mpath)], check=True)
    env = dict(os.environ, BFVM_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PINS],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert res.returncode != 0, f"mutant {name} survived the pins:\n{res.stdout[-2000:]}"
