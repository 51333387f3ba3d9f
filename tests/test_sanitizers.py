"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle (oracle/ewald.c) and the library's host-side plan precompute (the
operator builders, the lattice tensor of eq. 12, the interaction lists and
their symmetry folding, the matrix-core swizzles; csrc/harmonics_host.cpp and
csrc/m2l_layout.cpp) and the batch autotune cache file (csrc/tuning_cache.cpp)
are built with -fsanitize=address,undefined and driven over small inputs and
every order p the benchmarks use: any out-of-bounds
access, use after free, leak or undefined arithmetic aborts the driver.  No
GPU code is built or run here (the host files are compiled host-only).
"""
import os
import shutil
import subprocess
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2003_13218_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
# for hipcc: every sanitizer flag goes to the host pass only
HIP_SAN = [f for x in SAN for f in (("-Xarch_host", x) if "sanitize" in x else (x,))]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")

ORACLE_DRIVER = textwrap.dedent(r"""
    #include <math.h>
    #include <stdint.h>
    #include <stdio.h>
    #include <stdlib.h>
    int oracle_ewald(int64_t, const double *, const double *, double, double, double, double, int64_t,
                     const int64_t *, double *, double *, double *);
    int oracle_ewald_uv(int64_t, const double *, const double *, const uint8_t *, double, double, double, double,
                        double *);
    int oracle_nearfield(int64_t, const double *, const double *, double, int, int, double *, double *);
    int main(void) {
        const int64_t n = 40;
        double pos[120], q[40], terms[5], phi[40], f[120], uv[4], pn[40], fn[120];
        uint8_t mask[40];
        unsigned s = 12345u;
        for (int i = 0; i < 120; ++i) { s = s * 1103515245u + 12345u; pos[i] = 9.0 * (s >> 8) / 16777216.0 - 1.0; }
        for (int i = 0; i < 40; ++i) { q[i] = (i % 3 == 0) ? -0.8 : 0.4; mask[i] = i < 3; }
        int64_t idx[5] = {0, 7, 13, 21, 39};
        int rc = oracle_ewald(n, pos, q, 7.0, 0.8, 3.5, 4.0, n, NULL, terms, phi, f);
        rc |= oracle_ewald(n, pos, q, 7.0, 0.8, 3.5, 4.0, 5, idx, terms, phi, f);
        rc |= oracle_ewald_uv(n, pos, q, mask, 7.0, 0.8, 3.5, 4.0, uv);
        for (int lv = 1; lv <= 3; ++lv) rc |= oracle_nearfield(n, pos, q, 7.0, lv, 2, pn, fn);
        rc |= oracle_ewald(0, pos, q, 7.0, 0.8, 3.5, 4.0, 0, NULL, terms, phi, f);
        printf("oracle rc=%d E=%.10f\n", rc, terms[4]);
        return rc != 0;
    }
""")

HOST_DRIVER = textwrap.dedent(r"""
    #include "fmm_internal.h"
    #include <cstdio>
    #include <vector>
    using namespace fmm;
    int main() {
        Offsets o = build_offsets();
        int bad = 0;
        for (int p : {0, 1, 2, 4, 5, 8, 10, 12, 16, 20}) {
            const int K = num_coeffs(p);
            std::vector<int32_t> list((size_t)8 * m2l_list_entries(p) * m2l_list_width(p));
            if (!build_m2l_list(p, o.vec.data(), o.il.data(), list.data())) ++bad;
            std::vector<int32_t> map((size_t)16 * m2l_row_blocks(p));
            m2l_row_map(p, map.data());
            std::vector<double> ops((size_t)kNumOffsets * K * K, 0.0);
            for (int i = 0; i < kNumOffsets; i += (p > 12 ? 301 : 37)) {
                const double t[3] = {(double)o.vec[3 * i], (double)o.vec[3 * i + 1], (double)o.vec[3 * i + 2]};
                build_m2l_operator(p, t, ops.data() + (size_t)i * K * K);
            }
            std::vector<float> sw(m2l_ops_elems<float>(p));
            swizzle_m2l_ops<float>(p, ops.data(), sw.data());
            std::vector<uint16_t> bf(m2l_bf16_ops_elems(p));
            swizzle_m2l_ops_bf16(p, ops.data(), bf.data());
            std::vector<uint16_t> h16(m2l_split16_ops_elems(p));
            std::vector<float> sc((size_t)2 * padded_coeffs(p));
            swizzle_m2l_ops_split16(p, ops.data(), h16.data(), sc.data(), sc.data() + padded_coeffs(p));
            for (int k = 0; k < 2 * padded_coeffs(p); ++k)
                if (!(sc[k] > 0.0f)) ++bad;
            std::vector<cplx> T((size_t)(2 * p + 1) * (2 * p + 1));
            lattice_tensor(2 * p, 3.0, T.data());
            std::vector<double> A((size_t)K * K), tree((size_t)16 * K * K);
            build_lattice_operator(p, T.data(), A.data());
            for (int oc = 0; oc < 8; ++oc) {
                build_m2m_operator(p, oc, tree.data() + (size_t)oc * K * K);
                build_l2l_operator(p, oc, tree.data() + (size_t)(8 + oc) * K * K);
            }
            std::vector<double> s64((size_t)16 * padded_coeffs(p) * padded_coeffs(p));
            swizzle_ops<double>(p, 16, tree.data(), s64.data());
            RecTables rt;
            build_rec_tables(&rt);
        }
        std::printf("host precompute bad=%d\n", bad);
        return bad;
    }
""")


CACHE_DRIVER = textwrap.dedent(r"""
    #include "fmm_internal.h"
    #include <cstdio>
    #include <vector>
    using namespace fmm;
    int main(int argc, char **argv) {
        if (argc < 2) return 2;
        const char *path = argv[1];
        int bad = 0;
        const double box[3] = {30.5, 41.25, 52.0};
        const int64_t na[3] = {1000, 2500, 0}, nb[3] = {1000, 2501, 0};
        const std::string k = tuning_cache_key("gfx950:sramecc+ x\t", 10, 1, 3, 3, box, na);
        const std::string k2 = tuning_cache_key("gfx950:sramecc+ x\t", 10, 1, 3, 3, box, nb);
        if (k.find('\t') != std::string::npos || k.find(' ', 15) == std::string::npos || k == k2) ++bad;
        std::vector<int> lv, gr;
        if (tuning_cache_lookup(path, k, 3, lv, gr)) ++bad;  // no file yet
        FILE *fp = std::fopen(path, "wb");
        if (!fp) return 3;
        std::fprintf(fp, "foreign line\n\n%s\n", k.c_str());
        std::fprintf(fp, "%s\t3,3\t4,4,4\n", k.c_str());        // too few depths
        std::fprintf(fp, "%s\t3,11,3\t4,4,4\n", k.c_str());     // depth out of range
        std::fprintf(fp, "%s\t3,3,3\t4,5,4\n", k.c_str());      // not a group count
        std::fprintf(fp, "%s\t3,3,3,\t4,4,4\n", k.c_str());     // trailing comma
        std::fprintf(fp, "%sX\t3,3,3\t4,4,4\n", k.c_str());     // longer key
        std::fclose(fp);
        if (tuning_cache_lookup(path, k, 3, lv, gr)) ++bad;
        if (!tuning_cache_append(path, k, {3, 2, 4}, {4, 8, 0})) ++bad;
        if (!tuning_cache_lookup(path, k, 3, lv, gr) || lv != std::vector<int>{3, 2, 4} ||
            gr != std::vector<int>{4, 8, 0}) ++bad;
        if (tuning_cache_lookup(path, k2, 3, lv, gr)) ++bad;  // another batch
        if (!tuning_cache_append(path, k2, {1, 1, 1}, {16, 16, 16})) ++bad;
        if (!tuning_cache_append(path, k, {2, 2, 2}, {2, 2, 2})) ++bad;
        fp = std::fopen(path, "ab");
        if (!fp) return 3;
        std::fprintf(fp, "%s\t5,5,5\t16,16,16", k.c_str());  // torn append: no line feed
        std::fclose(fp);
        if (!tuning_cache_lookup(path, k, 3, lv, gr) || lv != std::vector<int>{2, 2, 2} ||
            gr != std::vector<int>{2, 2, 2}) ++bad;  // the last complete line wins
        if (!tuning_cache_lookup(path, k2, 3, lv, gr) || lv != std::vector<int>{1, 1, 1}) ++bad;
        if (tuning_cache_append("/nonexistent-dir/x/cache.txt", k, {1, 1, 1}, {0, 0, 0})) ++bad;
        std::printf("tuning cache bad=%d\n", bad);
        return bad;
    }
""")


def _run(cmd, env=None, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env or ENV, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    drv = tmp_path / "drv.c"
    drv.write_text(ORACLE_DRIVER)
    exe = tmp_path / "oracle_san"
    _run(["gcc", "-std=c99", "-fopenmp", *SAN, str(drv), os.path.join(ROOT, "oracle", "ewald.c"), "-o", str(exe),
          "-lm"])
    r = _run([str(exe)], timeout=120, env=dict(ENV, OMP_NUM_THREADS="2"))
    assert "oracle rc=0" in r.stdout


def test_host_precompute_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    drv = tmp_path / "drv.cpp"
    drv.write_text(HOST_DRIVER)
    objs = []
    for src in ("harmonics_host.cpp", "m2l_layout.cpp", str(drv)):
        path = src if os.path.isabs(src) else os.path.join(CSRC, src)
        obj = tmp_path / (os.path.basename(path) + ".o")
        # host-only compilation: each -fsanitize= goes to the host pass only
        _run([hipcc, "-x", "hip", "--cuda-host-only", "-std=c++17", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
              *HIP_SAN, "-c", path, "-o", str(obj)])
        objs.append(str(obj))
    exe = tmp_path / "host_san"
    _run([hipcc, *HIP_SAN, *objs, "-o", str(exe), "-lpthread"])
    r = _run([str(exe)], timeout=600)
    assert "host precompute bad=0" in r.stdout


def test_tuning_cache_under_sanitizers(tmp_path):
    # the autotune cache file of batch plans (csrc/tuning_cache.cpp): keys,
    # round trip, last line wins, foreign / malformed / torn lines skipped
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    drv = tmp_path / "cache_drv.cpp"
    drv.write_text(CACHE_DRIVER)
    objs = []
    for path in (os.path.join(CSRC, "tuning_cache.cpp"), str(drv)):
        obj = tmp_path / (os.path.basename(path) + ".o")
        _run([hipcc, "-x", "hip", "--cuda-host-only", "-std=c++17", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
              *HIP_SAN, "-c", path, "-o", str(obj)])
        objs.append(str(obj))
    exe = tmp_path / "cache_san"
    _run([hipcc, *HIP_SAN, *objs, "-o", str(exe), "-lpthread"])
    r = _run([str(exe), str(tmp_path / "autotune.txt")], timeout=120)
    assert "tuning cache bad=0" in r.stdout
