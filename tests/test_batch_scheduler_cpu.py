"""CPU check of the batched form's persistent single-launch scheduler, which
the library keeps switched off: the programs the library builds for the
96-domain workload (forward step and the 32-domain reverse step, three work
sizes per item) are checked for their dependency layout, then the kernel's
protocol (atomic queue head, per-stage counters, bounded waits, error flag,
release/acquire fences) is run by host threads standing in for resident
workgroups.  See tests/batch_sched_emu.cpp for the checks."""
import os
import shutil
import subprocess

import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_persistent_scheduler_protocol_is_deadlock_free(tmp_path):
    exe = str(tmp_path / "batch_sched_emu")
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-I", os.path.join(ROOT, "paper_2602_05017_amd", "csrc"),
                    "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "batch_sched_emu.cpp"), "-o", exe],
                   check=True)
    probs = workloads.batch_config(with_field=False)
    lines = []
    for k, p in enumerate(probs):
        nsrc = len(p.src) if p.src is not None else 0
        ndir = 16 if k % 5 == 1 else 0          # some domains with Dirichlet entries (every copy stage kept)
        if k % 7 == 3:
            nsrc = 0                             # and some with neither (no copy stage at all)
            ndir = 0
        lines.append(f"{p.nx} {p.ny} {p.nz} {p.S} {0 if p.dtype == 'f64' else 1} {nsrc} {ndir}")
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, timeout=900)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-2000:]
    assert "0 failed" in r.stdout
