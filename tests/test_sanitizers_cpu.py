"""Address and undefined-behaviour sanitizer runs of the host code (CPU only).

- The C oracle fill (oracle/csrc/efie_oracle.c) built with gcc
  -fsanitize=address,undefined, driven by a small C program on the level-1
  icosphere: no sanitizer report, and the matrix equals the regular build's.
- The library's host C++ (mesh.cpp: RWG table, validation, flagged pairs;
  rng.cpp: SplitMix64 + Floyd rows) built with ROCm's clang++ under the same
  sanitizers: valid and invalid meshes, row samples; results equal the
  oracle's.
Every sanitizer finding aborts the driver (-fno-sanitize-recover=all)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import cfill, sampling
from oracle.efie import Geometry
from oracle.mesh import flagged_pairs, rwg_table
from paper_2606_13482_amd.inputs import cube_sphere, icosphere

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
CLANG = "/opt/rocm/llvm/bin/clang++"

ORACLE_DRIVER = r"""
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>
void oracle_fill(int64_t F, int64_t N, int nq, const double *w, const double *X, const double *Vf,
                 const double *tri, const double *area, const int64_t *m_of, const double *s_of,
                 const uint8_t *flags, double k, int64_t ncol, const int64_t *cptr, const int64_t *ctris,
                 double *Z);
static void *slurp(const char *dir, const char *name, size_t *n) {
    char path[4096]; snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "rb"); if (!f) { perror(path); exit(2); }
    fseek(f, 0, SEEK_END); long sz = ftell(f); fseek(f, 0, SEEK_SET);
    void *p = malloc(sz > 0 ? sz : 1); if (fread(p, 1, sz, f) != (size_t)sz) exit(3); fclose(f);
    *n = (size_t)sz; return p;
}
int main(int argc, char **argv) {
    size_t n;
    int64_t *hdr = slurp(argv[1], "hdr", &n);     /* F, N, nq, ncol */
    double *k = slurp(argv[1], "k", &n);
    double *w = slurp(argv[1], "w", &n), *X = slurp(argv[1], "X", &n), *Vf = slurp(argv[1], "Vf", &n);
    double *tri = slurp(argv[1], "tri", &n), *area = slurp(argv[1], "area", &n), *s_of = slurp(argv[1], "s_of", &n);
    int64_t *m_of = slurp(argv[1], "m_of", &n), *cptr = slurp(argv[1], "cptr", &n), *ct = slurp(argv[1], "ctris", &n);
    uint8_t *flags = slurp(argv[1], "flags", &n);
    int64_t N = hdr[1];
    double *Z = calloc((size_t)(2 * N * N), sizeof(double));
    oracle_fill(hdr[0], N, (int)hdr[2], w, X, Vf, tri, area, m_of, s_of, flags, k[0], hdr[3], cptr, ct, Z);
    char path[4096]; snprintf(path, sizeof path, "%s/Z", argv[1]);
    FILE *f = fopen(path, "wb"); fwrite(Z, sizeof(double), (size_t)(2 * N * N), f); fclose(f);
    free(Z); free(hdr); free(k); free(w); free(X); free(Vf); free(tri); free(area); free(s_of); free(m_of);
    free(cptr); free(ct); free(flags);
    return 0;
}
"""

HOST_DRIVER = r"""
#include <cstdio>
#include <fstream>
#include <iterator>
#include <vector>
#include "bie_internal.hpp"
template <typename T> static std::vector<T> slurp(const std::string &p) {
    std::ifstream f(p, std::ios::binary);
    std::vector<char> b((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
    std::vector<T> v(b.size() / sizeof(T));
    if (!b.empty()) std::memcpy(v.data(), b.data(), b.size());
    return v;
}
int main(int argc, char **argv) {
    const std::string d = argv[1];
    auto V = slurp<double>(d + "/V");
    auto T = slurp<int32_t>(d + "/T");
    try {
        bie::Mesh m = bie::build_mesh(V.data(), int64_t(V.size() / 3), T.data(), int64_t(T.size() / 3), 2.0);
        std::ofstream e(d + "/edges", std::ios::binary);
        e.write(reinterpret_cast<const char *>(m.edges.data()), m.edges.size() * sizeof(int32_t));
        std::ofstream q(d + "/near", std::ios::binary);
        q.write(reinterpret_cast<const char *>(m.near.data()), m.near.size() * sizeof(int32_t));
        std::printf("ok %lld\n", (long long)m.N);
    } catch (const bie::Error &err) {
        std::printf("error %d %s\n", err.code, err.what());
    }
    auto rows = bie::rscc_rows(7680, 512, 1234);
    std::ofstream r(d + "/rows", std::ios::binary);
    r.write(reinterpret_cast<const char *>(rows.data()), rows.size() * sizeof(int64_t));
    return 0;
}
"""


def _run(cmd, **kw):
    p = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert p.returncode == 0, (cmd, p.stdout[-2000:], p.stderr[-4000:])
    return p.stdout


def test_oracle_fill_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    drv = tmp_path / "drv.c"
    drv.write_text(ORACLE_DRIVER)
    exe = tmp_path / "oracle_san"
    _run(["gcc", "-std=c11", *SAN, "-fopenmp", str(drv), os.path.join(ROOT, "oracle", "csrc", "efie_oracle.c"),
          "-o", str(exe), "-lm"])
    V, T = icosphere(1)
    rwg = rwg_table(V, T)
    k = 2.0
    G = Geometry(rwg)
    cols = cfill.colour_triangles(G.m_of)
    cptr = np.zeros(len(cols) + 1, np.int64)
    cptr[1:] = np.cumsum([c.size for c in cols])
    d = tmp_path / "in"
    d.mkdir()
    np.array([rwg["F"], rwg["N"], G.w.size, len(cols)], np.int64).tofile(d / "hdr")
    np.array([k]).tofile(d / "k")
    for name, arr, dt in (("w", G.w, np.float64), ("X", G.X, np.float64), ("Vf", G.Vf, np.float64),
                          ("tri", G.tri, np.float64), ("area", rwg["area"], np.float64),
                          ("s_of", G.s_of, np.float64), ("m_of", G.m_of, np.int64), ("cptr", cptr, np.int64),
                          ("ctris", np.concatenate(cols), np.int64),
                          ("flags", flagged_pairs(rwg, 2.0), np.uint8)):
        np.ascontiguousarray(arr, dt).tofile(d / name)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1")
    _run([str(exe), str(d)], env=env)
    Z = np.fromfile(d / "Z", np.float64).view(np.complex128).reshape(rwg["N"], rwg["N"])
    Zr = cfill.fill(rwg, k)
    assert np.max(np.abs(Z - Zr)) <= 1e-13 * np.max(np.abs(Zr))


@pytest.mark.parametrize("case", ["icosphere", "ellipsoid", "open", "misoriented", "zero_area"])
def test_host_mesh_and_rows_under_sanitizers(tmp_path, case):
    if not os.path.exists(CLANG):
        pytest.skip("ROCm clang++ not available")
    drv = tmp_path / "drv.cpp"
    drv.write_text(HOST_DRIVER.replace("#include <cstdio>", "#include <cstdio>\n#include <cstring>\n#include <string>"))
    exe = tmp_path / "host_san"
    csrc = os.path.join(ROOT, "paper_2606_13482_amd", "csrc")
    _run([CLANG, "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + csrc, str(drv),
          os.path.join(csrc, "mesh.cpp"), os.path.join(csrc, "rng.cpp"), "-o", str(exe)])
    if case == "ellipsoid":
        V, T = cube_sphere(4, "ellipsoid", axes=(1.0, 1.6, 2.3))
    else:
        V, T = icosphere(2)
    if case == "open":
        T = T[:-1]
    elif case == "misoriented":
        T = T.copy(); T[5] = T[5][[0, 2, 1]]
    elif case == "zero_area":
        V = V.copy(); V[T[3, 1]] = V[T[3, 0]]
    d = tmp_path / "in"
    d.mkdir()
    np.ascontiguousarray(V, np.float64).tofile(d / "V")
    np.ascontiguousarray(T, np.int32).tofile(d / "T")
    out = _run([str(exe), str(d)], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    rows = np.fromfile(d / "rows", np.int64)
    assert list(rows) == sampling.sample_rows(7680, 512, 1234)
    if case in ("icosphere", "ellipsoid"):
        assert out.startswith("ok")
        rwg = rwg_table(V, T)
        edges = np.fromfile(d / "edges", np.int32).reshape(-1, 4)
        assert np.array_equal(edges[:, 0:2], rwg["edges"]) and np.array_equal(edges[:, 2], rwg["tp"]) \
            and np.array_equal(edges[:, 3], rwg["tm"])
        near = np.fromfile(d / "near", np.int32).reshape(-1, 2)
        fl = flagged_pairs(rwg, 2.0)
        assert {(int(p), int(q)) for p, q in near} == {(int(p), int(q)) for p, q in zip(*np.nonzero(np.triu(fl)))}
    else:
        assert out.startswith("error -2"), out
