"""The library's host-side Hermitian eigensolver (csrc/herm_eig.h, cyclic Jacobi), used by the
Rayleigh-Ritz steps of the coarse deflation set-up: compiled with g++ and checked against
numpy's eigh on random, degenerate and indefinite matrices."""
import os
import subprocess

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <cstdio>
#include <complex>
#include <vector>
#include "herm_eig.h"
int main(int argc, char** argv) {
    FILE* f = std::fopen(argv[1], "rb");
    int m;
    if (std::fread(&m, sizeof(int), 1, f) != 1) return 1;
    std::vector<std::complex<double>> H((size_t)m * m), V((size_t)m * m);
    if (std::fread(H.data(), sizeof(double) * 2, (size_t)m * m, f) != (size_t)m * m) return 1;
    std::fclose(f);
    std::vector<double> lam(m);
    const int st = hdcr::herm_eig(m, H.data(), lam.data(), V.data());
    FILE* g = std::fopen(argv[2], "wb");
    std::fwrite(&st, sizeof(int), 1, g);
    std::fwrite(lam.data(), sizeof(double), m, g);
    std::fwrite(V.data(), sizeof(double) * 2, (size_t)m * m, g);
    std::fclose(g);
    return 0;
}
"""


def _run(tmp_path, exe, H):
    m = H.shape[0]
    inp, out = tmp_path / "h.bin", tmp_path / "v.bin"
    with open(inp, "wb") as f:
        f.write(np.int32(m).tobytes())
        f.write(np.ascontiguousarray(H, dtype=np.complex128).tobytes())
    subprocess.run([str(exe), str(inp), str(out)], check=True)
    raw = open(out, "rb").read()
    st = int(np.frombuffer(raw[:4], dtype=np.int32)[0])
    lam = np.frombuffer(raw[4:4 + 8 * m], dtype=np.float64)
    V = np.frombuffer(raw[4 + 8 * m:], dtype=np.complex128).reshape(m, m)
    return st, lam, V


def test_herm_eig_against_numpy(tmp_path):
    src = tmp_path / "drv.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "drv"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I" + os.path.join(ROOT, "paper_1611_06944_amd", "csrc"),
                    str(src), "-o", str(exe)], check=True)
    rng = np.random.default_rng(3)
    cases = []
    for m in (1, 2, 5, 16, 48, 64):
        X = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
        cases.append(0.5 * (X + X.conj().T))
    # degenerate: a unitary rotation of diag with repeated and +- paired values
    m = 12
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    d = np.array([-3.0, -3.0, -1.0, -1.0, 1.0, 1.0, 2.0, 2.0, 2.0, 5.0, 0.0, 0.0])
    cases.append(Q @ np.diag(d) @ Q.conj().T)
    for H in cases:
        st, lam, V = _run(tmp_path, exe, H)
        assert st >= 0
        scale = max(np.abs(H).max(), 1.0)
        np.testing.assert_allclose(lam, np.linalg.eigvalsh(H), atol=1e-12 * scale * H.shape[0])
        np.testing.assert_allclose(V.conj().T @ V, np.eye(H.shape[0]), atol=1e-12)
        np.testing.assert_allclose(H @ V, V * lam[None, :], atol=1e-11 * scale * H.shape[0])
