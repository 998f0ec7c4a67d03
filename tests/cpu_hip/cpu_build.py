"""Host-only build of libhigs's own HIP sources against the CPU stand-in
runtime in tests/cpu_hip/hip/ (AddressSanitizer on), plus a driver that
renders frames through the C-ABI.  Test infrastructure: the product library
is the gfx950 build of paper_2606_00352_amd/build.py.

run_frames() renders a scene for a list of cameras in a child process under a
time limit and returns what the driver wrote, so that a CPU test can check
every kernel's termination and memory accesses (ASan aborts the child on an
out-of-bounds access) and compare results with the oracle.
"""
from __future__ import annotations

import glob
import hashlib
import os
import shutil
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2606_00352_amd", "csrc")
BUILD = os.path.join(HERE, "_build")
DRIVER = os.path.join(BUILD, "frame_driver")

CXX = os.environ.get("CPUHIP_CXX", "/opt/rocm/lib/llvm/bin/clang++")
FLAGS = ["-std=c++20", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
         "-Wno-unknown-attributes", "-I", HERE]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


def available() -> bool:
    return shutil.which(CXX) is not None or os.path.exists(CXX)


def _inputs():
    files = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.h")))
    files += [os.path.join(HERE, "hip", "hip_runtime.h"), os.path.join(HERE, "frame_driver.cpp"),
              os.path.join(ROOT, "include", "higs.h")]
    h = hashlib.sha256()
    for f in files:
        with open(f, "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()


def build() -> str:
    """Compiles every .hip source for the host and links the driver (cached by
    a hash of the sources)."""
    os.makedirs(BUILD, exist_ok=True)
    stamp = os.path.join(BUILD, "stamp")
    key = _inputs()
    if os.path.exists(DRIVER) and os.path.exists(stamp) and open(stamp).read() == key:
        return DRIVER
    objs, procs = [], []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        procs.append(subprocess.Popen([CXX, *FLAGS, *SAN, "-x", "c++", "-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(obj)
    drv = os.path.join(BUILD, "frame_driver.o")
    procs.append(subprocess.Popen([CXX, *FLAGS, *SAN, "-c", os.path.join(HERE, "frame_driver.cpp"), "-o", drv],
                                  stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    errs = []
    for p in procs:
        out, _ = p.communicate()
        if p.returncode:
            errs.append(out.decode(errors="replace"))
    if errs:
        raise RuntimeError("CPU build failed:\n" + "\n".join(errs)[-6000:])
    subprocess.check_call([CXX, *SAN, *objs, drv, "-o", DRIVER, "-lpthread"])
    with open(stamp, "w") as f:
        f.write(key)
    return DRIVER


class Frame:
    pass


def run_frames(scene, cams, max_pairs, max_batches, sort_mode=1, batch_cap=1024, n_cus=2,
               entry=0, uses=None, timeout=600, workdir=None, precision=0, sh_format=0, chain=64, fuse=1):
    """Renders `scene` (numpy arrays) for each camera; returns a list of Frame
    with rc, n_visible, n_pairs, n_batches, overflow, image, T, and (when the
    frame did not overflow) sorted keys/ids and the batch table."""
    drv = build()
    work = workdir or tempfile.mkdtemp(prefix="higs_cpu_")
    os.makedirs(work, exist_ok=True)
    try:
        means, scales, quats, opac, sh = [np.ascontiguousarray(a, dtype=np.float32) for a in scene.arrays()]
        n = means.shape[0]
        for name, a in (("means", means), ("scales", scales), ("quats", quats), ("opac", opac), ("sh", sh)):
            a.tofile(os.path.join(work, name))
        uses = uses or [n] * len(cams)
        with open(os.path.join(work, "job.txt"), "w") as f:
            f.write(f"{n} {max_pairs} {max_batches} {sort_mode} {batch_cap} {n_cus} {entry} {precision} "
                    f"{sh_format} {chain} {fuse}\n")
            for c, u in zip(cams, uses):
                w = np.asarray(c.world_to_cam, np.float32).reshape(-1)
                bg = getattr(c, "background", (0.0, 0.0, 0.0))
                vals = [u, c.width, c.height, *(repr(float(np.float32(v))) for v in (c.fx, c.fy, c.cx, c.cy))]
                vals += [repr(float(v)) for v in w] + [repr(float(np.float32(v))) for v in bg]
                f.write(" ".join(str(v) for v in vals) + "\n")
        out = os.path.join(work, "out")
        os.makedirs(out, exist_ok=True)
        env = dict(os.environ, CPUHIP_CUS=str(n_cus), ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
        r = subprocess.run([drv, work, out], env=env, capture_output=True, text=True, timeout=timeout)
        if r.returncode != 0:
            raise RuntimeError(f"frame driver failed ({r.returncode}):\n{r.stderr[-8000:]}")
        frames = []
        packed = None
        if os.path.exists(os.path.join(out, "packed")):
            packed = np.fromfile(os.path.join(out, "packed"), np.uint8)
        lines = open(os.path.join(out, "counts.txt")).read().split("\n")
        for k, c in enumerate(cams):
            fr = Frame()
            rc, vis, pairs, batches, evals, ovf, graphs = (int(x) for x in lines[k].split())
            fr.graphs = graphs
            fr.rc, fr.n_visible, fr.n_pairs, fr.n_batches, fr.overflow = rc, vis, pairs, batches, ovf
            fr.n_evaluations = evals
            fr.packed = packed
            pre = os.path.join(out, f"f{k}_")
            fr.image = np.fromfile(pre + "image", np.float32).reshape(c.height, c.width, 3)
            fr.T = np.fromfile(pre + "T", np.float32).reshape(c.height, c.width)
            fr.keys = fr.ids = fr.batches = None
            if os.path.exists(pre + "sorted"):
                raw = np.fromfile(pre + "sorted", np.uint8)
                npairs = raw.size // 12
                fr.keys = raw[:npairs * 8].view(np.uint64)
                fr.ids = raw[npairs * 8:].view(np.uint32)
            if os.path.exists(pre + "batches"):
                fr.batches = np.fromfile(pre + "batches", np.uint32).reshape(-1, 3)
            frames.append(fr)
        return frames
    finally:
        if workdir is None:
            shutil.rmtree(work, ignore_errors=True)
