"""The oracle's pins catch plausible mistakes (CPU only).

Each case below edits a copy of the oracle's C source with one mistake of the kind a
careful reader could still make (a wrong sign, index, factor or axis, a dropped term),
compiles it into a library of its own and runs the pin tests against it in a separate
process: at least one pin must fail.  The oracle itself is never modified.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

# (name, file, [(text, replacement), ...]); every text occurs exactly once in the file
SAL_MUTANTS = [
    ("reflection repeats the edge sample", "sal_oracle.c",
     [("    if (u < 0) return -u;\n    if (u >= n) return 2 * (n - 1) - u;\n    return u;\n}\n\n/* Signed",
       "    if (u < 0) return -u - 1;\n    if (u >= n) return 2 * n - 1 - u;\n    return u;\n}\n\n/* Signed")]),
    ("window starts one sample late along t", "sal_oracle.c",
     [("long a = refl_index(t - h + p, n0);", "long a = refl_index(t - h + 1 + p, n0);")]),
    ("DFT exponent of the wrong sign", "sal_oracle.c",
     [("sw[k] = -sin(2.0 * M_PI * (double)k / (double)L);", "sw[k] = sin(2.0 * M_PI * (double)k / (double)L);")]),
    ("1/L^3 of the DFT dropped", "sal_oracle.c",
     [("F[2 * o] = re / (double)L3;\n                F[2 * o + 1] = im / (double)L3;",
       "F[2 * o] = re;\n                F[2 * o + 1] = im;")]),
    ("x twiddle index transposed", "sal_oracle.c",
     [("double c = cw[q * nu % L], s = sw[q * nu % L];", "double c = cw[(q + nu) % L], s = sw[(q + nu) % L];")]),
    ("unsigned frequencies in the projections", "sal_oracle.c",
     [("return (u <= L / 2) ? u : u - L;", "return u;")]),
    ("projection onto the wrong plane for E_t", "sal_oracle.c",
     [("acc[0] += mag * sqrt(j * j + k * k) / rho;", "acc[0] += mag * sqrt(i * i + k * k) / rho;")]),
    ("magnitude without the imaginary part", "sal_oracle.c",
     [("double mag = sqrt(F[2 * o] * F[2 * o] + F[2 * o + 1] * F[2 * o + 1]);", "double mag = fabs(F[2 * o]);")]),
    ("mean over L^3 bins, DC counted", "sal_oracle.c",
     [("double nbins = (double)(L * L * L - 1);", "double nbins = (double)(L * L * L);")]),
    ("energies of x and y stored swapped", "sal_oracle.c",
     [("E[nb + v] = e[1];\n            E[2 * nb + v] = e[2];", "E[nb + v] = e[2];\n            E[2 * nb + v] = e[1];")]),
    ("Eq. (5) weight on the centre instead of the neighbour", "sal_oracle.c",
     [("sum += fabs(centre - w * nbv);", "sum += fabs(w * centre - nbv);")]),
    ("Gaussian without the factor 2", "sal_oracle.c",
     [("double w = exp(-(double)(s * s * len2) / (2.0 * sigma * sigma));",
       "double w = exp(-(double)(s * s * len2) / (sigma * sigma));")]),
    ("Q counts rays, not samples", "sal_oracle.c",
     [("double Q = (double)(nrays * r);", "double Q = (double)(nrays);")]),
    ("rays one sample short", "sal_oracle.c",
     [("for (long s = 1; s <= r; ++s) {\n                    long rel[3];", "for (long s = 1; s < r; ++s) {\n                    long rel[3];")]),
    ("anti-diagonal rays of a plane swapped", "sal_oracle.c",
     [("static const int sg[4][2] = {{1, 1}, {-1, -1}, {1, -1}, {-1, 1}};",
       "static const int sg[4][2] = {{1, 1}, {-1, -1}, {-1, 1}, {1, -1}};")]),
    ("normalisation without the minimum", "sal_oracle.c",
     [("s += abc[m] * (normalize ? (x - lo[m]) * scale[m] : x);", "s += abc[m] * (normalize ? x * scale[m] : x);")]),
    ("normalisation by the maximum alone", "sal_oracle.c",
     [("scale[m] = (hi[m] - lo[m] > zero_range * vmax) ? 1.0 / (hi[m] - lo[m]) : 0.0;",
       "scale[m] = (hi[m] - lo[m] > zero_range * vmax) ? 1.0 / hi[m] : 0.0;")]),
    ("lattice interpolation over s + 1 samples", "sal_oracle.c",
     [("f[a] = k1[a] == k0[a] ? 0.0 : (double)(pos[a] - k0[a] * s) / (double)s;",
       "f[a] = k1[a] == k0[a] ? 0.0 : (double)(pos[a] - k0[a] * s) / (double)(s + 1);")]),
]

NET_MUTANTS = [
    ("GELU with 1 - erf", "net_oracle.c",
     [("double oracle_gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }",
       "double oracle_gelu(double z) { return 0.5 * z * (1.0 - erf(z / sqrt(2.0))); }")]),
    ("GELU derivative with the wrong normal density", "net_oracle.c",
     [("z * exp(-0.5 * z * z) / sqrt(2.0 * M_PI);", "z * exp(-0.5 * z * z) / sqrt(M_PI);")]),
    ("forward taps mirrored along w", "net_oracle.c",
     [("                                       ww = nrefl(w + k % 3 - 1, S);\n                            const double *xp",
       "                                       ww = nrefl(w - k % 3 + 1, S);\n                            const double *xp")]),
    ("bias ignored", "net_oracle.c",
     [("double acc = bias ? bias[co] : 0.0;", "double acc = 0.0;")]),
    ("input gradient with the flipped kernel", "net_oracle.c",
     [("if (dx) dx[xo + ci] += g * W[(co * 27 + k) * ci_n + ci];",
       "if (dx) dx[xo + ci] += g * W[(co * 27 + (26 - k)) * ci_n + ci];")]),
]


def _build_mutant(tmp_path, fname, edits):
    srcs = {}
    for f in ("sal_oracle.c", "net_oracle.c"):
        with open(os.path.join(ORACLE, f)) as fh:
            srcs[f] = fh.read()
    for text, repl in edits:
        assert srcs[fname].count(text) == 1, text
        srcs[fname] = srcs[fname].replace(text, repl)
    paths = []
    for f, src in srcs.items():
        p = tmp_path / f
        p.write_text(src)
        paths.append(str(p))
    lib = str(tmp_path / "libmutant.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", lib] + paths + ["-lm"])
    return lib


def _pins_fail(lib, test_file):
    env = dict(os.environ, SAL_ORACLE_MUTANT_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", test_file)],
                       cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True, timeout=900)
    return r.returncode, r.stdout[-1500:]


@pytest.mark.parametrize("name,fname,edits", SAL_MUTANTS, ids=[m[0] for m in SAL_MUTANTS])
def test_saliency_pins_catch(tmp_path, name, fname, edits):
    rc, out = _pins_fail(_build_mutant(tmp_path, fname, edits), "test_oracle_pins.py")
    # pytest exit code 1: some tests failed (0 would mean every pin passed)
    assert rc == 1, (name, rc, out)


@pytest.mark.parametrize("name,fname,edits", NET_MUTANTS, ids=[m[0] for m in NET_MUTANTS])
def test_net_pins_catch(tmp_path, name, fname, edits):
    rc, out = _pins_fail(_build_mutant(tmp_path, fname, edits), "test_oracle_net.py")
    assert rc == 1, (name, rc, out)


def test_unmodified_copy_passes(tmp_path):
    """The harness itself: an unmodified copy compiled the same way passes every pin."""
    lib = _build_mutant(tmp_path, "sal_oracle.c", [])
    for f in ("test_oracle_pins.py", "test_oracle_net.py"):
        rc, out = _pins_fail(lib, f)
        assert rc == 0, (f, out)
