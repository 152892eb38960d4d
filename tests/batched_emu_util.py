"""Build and run the host emulation of the batched persistent kernel
(tests/emu): the kernel's own source compiled for the CPU with
AddressSanitizer, one emulated 256-work-item workgroup at a time.  Test
infrastructure only."""
from __future__ import annotations

import os
import struct
import subprocess
import tempfile
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.path.join(HERE, "emu")
CSRC = os.path.join(os.path.dirname(HERE), "paper_2310_09417_amd", "csrc")
CLANG = os.environ.get("RID_EMU_CXX", "/opt/rocm/llvm/bin/clang++")


def build(out_dir: str) -> str:
    exe = os.path.join(out_dir, "batched_emu")
    cmd = [CLANG, "-std=c++17", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
           "-Wno-psabi", "-Wno-pass-failed", "-I", EMU, "-I", CSRC, "-o", exe,
           os.path.join(EMU, "batched_emu.cpp"), os.path.join(EMU, "emu_sched.cpp")]
    subprocess.check_call(cmd)
    return exe


@dataclass
class EmuOut:
    k: np.ndarray
    status: np.ndarray
    passes: np.ndarray
    err_est: np.ndarray
    J: list
    T: list


def run(exe: str, blocks, b: int, tol: float, seed: int, dtype=np.float64, kmax=None, hints=None,
        order=None, relative=True, groups: int = 2, gap: int = 1 << 16, max_n=None,
        max_kmax=None, timeout=1200, factor=None, threads: int = 256) -> EmuOut:
    """dtype: storage type of the blocks; factor: np.float64 with float32
    blocks runs the FP32-storage, FP64-factorisation instantiation."""
    nblk = len(blocks)
    ms = [int(a.shape[0]) for a in blocks]
    ns = [int(a.shape[1]) for a in blocks]
    if kmax is None:
        kmax = [min(a, c) for a, c in zip(ms, ns)]
    elif isinstance(kmax, int):
        kmax = [kmax] * nblk
    caps = [min(k, a, c) for k, a, c in zip(kmax, ms, ns)]
    max_n = max(ns) if max_n is None else max_n
    max_kmax = max(caps) if max_kmax is None else max_kmax
    if factor is not None and factor != dtype:
        assert factor == np.float64 and dtype == np.float32
        dt = 2
    else:
        dt = 0 if dtype == np.float64 else 1
    tdtype = np.float64 if dt != 1 else np.float32
    with tempfile.TemporaryDirectory() as td:
        fin, fout = os.path.join(td, "in.bin"), os.path.join(td, "out.bin")
        with open(fin, "wb") as f:
            f.write(struct.pack("<10i", dt, nblk, b, 1 if relative else 0, max_n, max_kmax, groups,
                                1 if hints is not None else 0, 1 if order is not None else 0,
                                threads))
            f.write(struct.pack("<dQQ", tol, seed, gap))
            for i in range(nblk):
                h = int(hints[i]) if hints is not None else 0
                f.write(struct.pack("<4i", ms[i], ns[i], int(kmax[i]), h))
            if order is not None:
                f.write(np.asarray(order, dtype="<i4").tobytes())
            for a in blocks:
                f.write(np.ascontiguousarray(a, dtype=dtype).tobytes())
        env = dict(os.environ)
        env["ASAN_OPTIONS"] = "detect_leaks=0:detect_stack_use_after_return=0:abort_on_error=1"
        r = subprocess.run([exe, fin, fout], env=env, capture_output=True, text=True,
                           timeout=timeout)
        if r.returncode != 0:
            raise RuntimeError(f"batched_emu failed ({r.returncode}):\n{r.stderr[-6000:]}")
        data = open(fout, "rb").read()
    es = np.dtype(tdtype).itemsize
    off = 0
    ks, sts, ps, Es, Js, Ts = [], [], [], [], [], []
    for i in range(nblk):
        k, st, p = struct.unpack_from("<3i", data, off)
        off += 12
        (E,) = struct.unpack_from("<d", data, off)
        off += 8
        kk = max(k, 0)
        J = np.frombuffer(data, dtype="<i4", count=kk, offset=off).copy()
        off += 4 * kk
        nt = kk * (ns[i] - kk)
        T = np.frombuffer(data, dtype=tdtype, count=nt, offset=off).reshape(kk, ns[i] - kk).copy()
        off += es * nt
        ks.append(k), sts.append(st), ps.append(p), Es.append(E), Js.append(J), Ts.append(T)
    return EmuOut(np.array(ks), np.array(sts), np.array(ps), np.array(Es), Js, Ts)
