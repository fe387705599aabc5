"""Index maps of the step kernels, checked on the CPU (no GPU).

tests/emu/tile_emu.cpp compiles the library's device functions (lbm_device.h) for the host and
runs every workgroup of the fused single step, the two-steps-per-launch tiles (64x8, 64x4,
128x4, 64x16, interior and edge variants), the psi pass and the per-node observables with
poisoned memory (NaN in every slot that is not state, NaN in the LDS before each tile), under
AddressSanitizer and UndefinedBehaviorSanitizer. It fails when a launch reads outside its
buffers, reads an LDS slot not written in the same launch, writes outside the state, or when the
two-step tiles differ by one bit from two fused steps. On periodic and bounce-back lattices the
adjoint's kernels run too: the segment recomputation (two steps with the intermediate state
written) must equal two fused steps, and a reverse step must write all of its outputs on the
fluid nodes only, bit-equal between the generic tile everywhere and 32x4 and 64x4 tiles that
take the interior variant where it applies. Lattices from 3x4 to 125x17 (ragged
tiles, halo wraps) and two with interior tiles; periodic, bounce-back (with and without ghost
rows), wet-node and solid-mask geometries; both equations of state.

The checker is itself checked: copies of the header with an index mistake planted must fail.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "emu", "tile_emu.cpp")
HEADER = os.path.join(ROOT, "paper_1410_2569_amd", "csrc", "lbm_device.h")
CXX = os.environ.get("CXX_EMU", "/opt/rocm/llvm/bin/clang++")
BASE = ["-std=c++20", "-O0", "-g", "-pthread", "-w", "-I", os.path.join(HERE, "emu")]

pytestmark = pytest.mark.skipif(not shutil.which(CXX), reason=f"{CXX} not available")


def _build(out, extra=()):
    subprocess.check_call([CXX, *BASE, *extra, SRC, "-o", out])
    return out


def test_index_maps_under_sanitizers(tmp_path):
    exe = _build(str(tmp_path / "tile_emu"),
                 ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=900,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "passed: 0 failure(s)" in r.stdout
    assert r.stdout.count("\nok ") + r.stdout.startswith("ok ") >= 40


@pytest.mark.parametrize("old,new,case", [
    # the last slot of the outer psi ring of the two-step tile never written
    ("h < NRING; h += NT", "h < NRING - 1; h += NT", ("65", "13", "1", "1", "0", "2")),
    # ... the same where a thread issues both of its pulls before either psi (64 x 8 on 512 threads)
    ("} else if (h >= 0 && h < NRING) {", "} else if (h >= 0 && h < NRING - 1) {",
     ("65", "13", "1", "1", "0", "2")),
    # the last slot of the psi ring around the output tile never written
    ("h < NRING1; h += NT", "h < NRING1 - 1; h += NT", ("130", "30", "0", "1", "0", "0")),
    # a diagonal population pulled from the wrong column
    ("f[6] = bot ? (g + 8 * pl)[r0 + ux] : (g + 6 * pl)[rm + xp];",
     "f[6] = bot ? (g + 8 * pl)[r0 + ux] : (g + 6 * pl)[rm + ux];", ("33", "10", "1", "1", "1", "1")),
], ids=["psi_ring_R3", "psi_ring_R3_fused", "psi_ring_R1", "pull_column"])
def test_checker_catches_planted_index_mistakes(tmp_path, old, new, case):
    src = open(HEADER).read()
    assert src.count(old) == 1, old
    hdr = tmp_path / "lbm_device.h"
    hdr.write_text(src.replace(old, new))
    exe = _build(str(tmp_path / "tile_emu_mutant"), [f'-DLBM_DEVICE_HEADER="{hdr}"'])
    r = subprocess.run([exe, *case], capture_output=True, text=True, timeout=300)
    assert r.returncode != 0 and "FAIL" in r.stdout + r.stderr, r.stdout
