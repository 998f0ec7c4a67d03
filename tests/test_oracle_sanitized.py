"""The oracle's C code (forward and adjoint) run under AddressSanitizer and
UndefinedBehaviorSanitizer: a child process preloads their runtimes and loads
a sanitised build of the oracle (HIGS_ORACLE_SANITIZE=1), renders small frames
with every stage, their adjoint and the one-pixel definition, and must end
without a report; its image must equal the plain build's bit for bit."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys, numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
from paper_2606_00352_amd import scenes
assert oracle.build().endswith("liboracle_san.so")
sc, cams = scenes.config0()
cam = cams[0]
fr = oracle.frame(sc, cam)
prm = oracle.Params()
prm.batch_cap = 64
fr2 = oracle.frame(sc, cam, prm)
# ragged image, culled and edge gaussians
sc3 = scenes.clustered_scene(3000, seed=5, n_clusters=4)
cam3 = scenes.orbit_cameras(3, 7, 203, 97, 120.0)[1]
fr3 = oracle.frame(sc3, cam3)
rng = np.random.default_rng(9)
small = scenes.clustered_scene(400, seed=6, n_clusters=2)
camg = scenes.orbit_cameras(2, 3, 96, 64, 80.0)[0]
dimg = rng.uniform(-1, 1, (camg.height, camg.width, 3))
_, dgeo, grads = oracle.frame_grad(small, camg, dimg, rng.uniform(-1, 1, (camg.height, camg.width)))
pix = np.array([[5, 7], [100, 200], [255, 0]])
oracle.render_untiled(fr.valid, fr.geo, cam, pixels=pix)
oracle.render_signature(fr.geo, fr.sorted_gid, fr.batch_tab, cam)
np.save(sys.argv[2], fr.image)
print("ok", fr.image.shape, int(fr2.batch_tab.shape[0]), float(np.abs(dgeo).sum()) > 0)
"""


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc's sanitizer runtimes are not installed")
    import oracle
    from paper_2606_00352_amd import scenes
    env = dict(os.environ, HIGS_ORACLE_SANITIZE="1", LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    out = tmp_path / "img.npy"
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, str(out)], env=env, capture_output=True,
                       text=True, timeout=900)
    report = r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
    assert r.stdout.startswith("ok"), r.stdout
    sc, cams = scenes.config0()
    assert np.array_equal(np.load(out), oracle.frame(sc, cams[0]).image)
