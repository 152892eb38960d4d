"""The Schur-update kernel's own source (rid_schur.hpp) executed on the CPU in
the workgroup emulation under AddressSanitizer, against the same product
formed by NumPy: S = Z(non-pivots, block) - Z(non-pivots, K) U2(K, block) in
place, pivot rows untouched, and the FP64 sums of S^2 per workgroup, for
the K ranges, column groups and tile counts the library launches
(including a K range that starts at kb, ragged K and ragged row counts).
The split-K form (k_schur_sk's FP64 partials per K range, summed in split
order and subtracted by k_schur_fin) is checked the same way, and so is its
FP32 form on the BF16 matrix cores (k_schur_skb)."""
import os
import struct
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.path.join(HERE, "emu")
CSRC = os.path.join(os.path.dirname(HERE), "paper_2310_09417_amd", "csrc")
CLANG = os.environ.get("RID_EMU_CXX", "/opt/rocm/llvm/bin/clang++")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("schur") / "schur_emu")
    subprocess.check_call([CLANG, "-std=c++17", "-O1", "-g", "-fsanitize=address",
                           "-fno-omit-frame-pointer", "-Wno-psabi", "-Wno-pass-failed", "-I", EMU,
                           "-I", CSRC, "-o", out, os.path.join(EMU, "schur_emu.cpp"),
                           os.path.join(EMU, "emu_sched.cpp")])
    return out


def _run(exe, Z, U2T, pos, k, kb, zcol, w, nt, cg, frm, dtype, ksplit=0, bf=False):
    n, ldz = Z.shape
    ldu = U2T.shape[1]
    with tempfile.TemporaryDirectory() as td:
        fin, fout = os.path.join(td, "in"), os.path.join(td, "out")
        with open(fin, "wb") as f:
            f.write(struct.pack("<12i", 0 if dtype == np.float64 else 1, n, ldz, k, kb, zcol, w,
                                ldu, nt, 1 if frm else 0, cg, 1))
            f.write(np.ascontiguousarray(Z, dtype=dtype).tobytes())
            f.write(np.ascontiguousarray(U2T, dtype=dtype).tobytes())
            f.write(np.asarray(pos, dtype="<i4").tobytes())
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
        cmd = [exe, fin, fout] + ([str(ksplit)] if ksplit else []) + (["bf"] if bf else [])
        r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-4000:]
        data = open(fout, "rb").read()
    es = np.dtype(dtype).itemsize
    Zo = np.frombuffer(data, dtype=dtype, count=n * ldz).reshape(n, ldz).copy()
    norm = np.frombuffer(data, dtype=np.float64, offset=n * ldz * es)
    return Zo, norm


# (n, k, kb, w, nt, cg) as the library picks them: w <= 64, cg by row count
CASES = [(300, 100, 0, 64, 1, 4), (1200, 257, 0, 64, 1, 4), (700, 130, 0, 64, 2, 2),
         (130, 64, 0, 48, 3, 1), (900, 200, 0, 64, 4, 1), (500, 77, 0, 16, 1, 1),
         (400, 150, 37, 16, 1, 1), (333, 90, 64, 8, 1, 1)]


# split-K: (n, k, w, nt, cg, ksplit), splits on multiples of 64, a ragged last
# split, and the column tiles and row groups of the library's launches
SK_CASES = [(300, 256, 64, 4, 4, 128), (1000, 300, 64, 4, 1, 128), (517, 400, 48, 3, 2, 192),
            (200, 129, 16, 1, 4, 64), (700, 640, 33, 3, 1, 256)]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n,k,w,nt,cg,ksplit", SK_CASES)
def test_split_k_schur_matches_numpy(exe, dtype, n, k, w, nt, cg, ksplit):
    _check(exe, dtype, n, k, 0, w, nt, cg, ksplit)


@pytest.mark.parametrize("n,k,w,nt,cg,ksplit", SK_CASES)
def test_split_k_schur_bf16_split_matches_numpy(exe, n, k, w, nt, cg, ksplit):
    """The FP32 split-K product on the BF16 matrix cores (three-part split of
    both operands, six partial products): within the same FP32 bound."""
    _check(exe, np.float32, n, k, 0, w, nt, cg, ksplit, bf=True)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n,k,kb,w,nt,cg", CASES)
def test_schur_kernel_matches_numpy(exe, dtype, n, k, kb, w, nt, cg):
    _check(exe, dtype, n, k, kb, w, nt, cg, 0)


def _check(exe, dtype, n, k, kb, w, nt, cg, ksplit, bf=False):
    rng = np.random.default_rng(n + k + w)
    zcol = k
    ldz = ((k + w + 3) // 4) * 4
    ldu = ((k + 15) // 16) * 16
    Z = rng.standard_normal((n, ldz)).astype(dtype)
    U2T = np.zeros((w, ldu), dtype=dtype)
    U2T[:, :k] = rng.standard_normal((w, k))
    pos = -np.ones(n, dtype=np.int64)
    piv = rng.choice(n, size=k, replace=False)
    pos[piv] = np.arange(k)
    Zo, norm = _run(exe, Z, U2T, pos, k, kb, zcol, w, nt, cg, kb > 0, dtype, ksplit, bf)
    Z64 = Z.astype(np.float64)
    rows = pos < 0
    K = slice(kb, k)
    S = Z64[rows, zcol:zcol + w] - Z64[rows][:, K] @ U2T.astype(np.float64)[:, K].T
    u = 2.0 ** -53 if dtype == np.float64 else 2.0 ** -24
    scale = np.abs(Z64[rows][:, K]) @ np.abs(U2T.astype(np.float64)[:, K]).T + \
        np.abs(Z64[rows, zcol:zcol + w])
    assert np.all(np.abs(Zo[rows, zcol:zcol + w] - S) <= 8 * u * np.sqrt(k) * scale + 1e-300)
    # pivot rows and the columns outside the block are untouched
    assert np.array_equal(Zo[~rows], Z[~rows])
    assert np.array_equal(Zo[:, :zcol], Z[:, :zcol])
    assert np.array_equal(Zo[:, zcol + w:], Z[:, zcol + w:])
    # FP64 sums of S^2 per workgroup: their total is ||S||_F^2 of the stored S
    Ss = Zo[rows, zcol:zcol + w].astype(np.float64)
    assert abs(norm.sum() - (Ss ** 2).sum()) <= 1e-12 * (Ss ** 2).sum()
