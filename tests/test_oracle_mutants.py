"""The oracle's pins catch plausible mistakes: each case plants one mistake (a flipped sign, a
dropped term or pixel, a transposed operand, an off-by-one, a wrong constant) in a copy of the
oracle -- the C oracle rebuilt with gcc, or a Python module of the oracle package in a copy of
the test tree -- and runs the pin tests against that copy in a fresh process. The run must fail;
the unchanged copy must pass. Nothing here touches a GPU or the HIP library."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
PINS = "tests/test_oracle_pins.py"
SMOOTH = ["tests/test_oracle_ext_pins.py", "tests/test_oracle_refine_pins.py"]
NO_PHILOX = ["-k", "not philox"]  # the rocRAND cross-check builds a helper with hipcc; other pins suffice

# (name, source file, exact text, replacement, pin files, extra pytest arguments)
MUTANTS = [
    ("phase sign (Re[exp(-i phi) p])", "stt_oracle.c",
     "double term = cos(phi) * p_re - sin(phi) * p_im; /* Re[e^{i phi} p] */",
     "double term = cos(phi) * p_re + sin(phi) * p_im; /* Re[e^{i phi} p] */", [PINS], NO_PHILOX),
    ("last pixel dropped", "stt_oracle.c",
     "    for (int32_t k = 0; k < N; ++k) {\n        int64_t t = tr->t0 + k, r = rows[k];\n        int64_t e = t * m->ld + r;\n        double sg = m->sigma[e];\n        double p_re = m->Y[2 * e] / sg, p_im = m->Y[2 * e + 1] / sg;\n        double turns",
     "    for (int32_t k = 0; k < N - 1; ++k) {\n        int64_t t = tr->t0 + k, r = rows[k];\n        int64_t e = t * m->ld + r;\n        double sg = m->sigma[e];\n        double p_re = m->Y[2 * e] / sg, p_im = m->Y[2 * e + 1] / sg;\n        double turns",
     [PINS], NO_PHILOX),
    ("normalisation by sqrt(N - 1)", "stt_oracle.c",
     "    free(rows);\n    double S = s + c;\n    return norm == 1 ? S / (double)N : S / sqrt((double)N);\n}\n\n/* score tracks",
     "    free(rows);\n    double S = s + c;\n    return norm == 1 ? S / (double)N : S / sqrt((double)(N - 1));\n}\n\n/* score tracks",
     [PINS], NO_PHILOX),
    ("sigma multiplied instead of divided", "stt_oracle.c",
     "        double p_re = m->Y[2 * e] / sg, p_im = m->Y[2 * e + 1] / sg;\n        double turns",
     "        double p_re = m->Y[2 * e] * sg, p_im = m->Y[2 * e + 1] * sg;\n        double turns", [PINS], NO_PHILOX),
    ("control frequencies f0 and f2 transposed in Eq. 6", "stt_oracle.c",
     "uint64_t num = a * a * tr->f0 + 2 * a * b * tr->f1 + b * b * tr->f2;",
     "uint64_t num = a * a * tr->f2 + 2 * a * b * tr->f1 + b * b * tr->f0;", [PINS], NO_PHILOX),
    ("row rounded to nearest instead of floored", "stt_oracle.c",
     "rows[k] = (int32_t)(num / den);", "rows[k] = (int32_t)((num + den / 2) / den);", [PINS], NO_PHILOX),
    ("phase taken at the next row's frequency", "stt_oracle.c",
     "double turns = orc_phase_turns((int64_t)m->fq4_lo + r * m->dfq4, tr->dtau);",
     "double turns = orc_phase_turns((int64_t)m->fq4_lo + (r + 1) * m->dfq4, tr->dtau);", [PINS], NO_PHILOX),
    ("Philox key words transposed", "stt_oracle.c",
     "uint32_t n0 = hi1 ^ c1 ^ k0;", "uint32_t n0 = hi1 ^ c1 ^ k1;", [PINS], []),
    ("Philox Weyl constant off by one", "stt_oracle.c",
     "k1 += 0xBB67AE85u;", "k1 += 0xBB67AE86u;", [PINS], []),
    ("extent unranked with start and end order reversed", "stt_oracle.c",
     "    *t0 = (int32_t)a;\n", "    *t0 = (int32_t)(e - a);\n", [PINS], NO_PHILOX),
    ("delay not centred on zero", "stt_oracle.c",
     "tr->dtau = (int32_t)(-(int64_t)D + (int64_t)scale_u64(u2, 2 * (uint64_t)D + 1));",
     "tr->dtau = (int32_t)((int64_t)scale_u64(u2, 2 * (uint64_t)D + 1));", [PINS], NO_PHILOX),
    ("free t_mid: sign of c in the discriminant", "stt_oracle.c",
     "int64_t D = b * b - 4 * a * c, U = 2 * a * (a * f0 - C * c) - b * V;",
     "int64_t D = b * b + 4 * a * c, U = 2 * a * (a * f0 - C * c) - b * V;", ["tests/test_oracle_tmid_pins.py"], []),
    ("free t_mid: t1 taken as the midpoint's mirror", "stt_oracle.c",
     "int64_t a = (int64_t)tr->t0 - 2 * (int64_t)tr->t1 + tr->t2, b = 2 * ((int64_t)tr->t1 - tr->t0);",
     "int64_t a = (int64_t)tr->t0 - 2 * (int64_t)tr->t1 + tr->t2, b = 2 * ((int64_t)tr->t2 - tr->t1);",
     ["tests/test_oracle_tmid_pins.py"], []),
    ("delay grid: ties to the highest delay index", "stt_oracle.c",
     "if (bm < 0 || z > best) { best = z; bm = k; }", "if (bm < 0 || z >= best) { best = z; bm = k; }",
     ["tests/test_oracle_maxdelay_pins.py"], []),
    ("delay grid: last delay of the grid skipped", "stt_oracle.c",
     "    for (int32_t k = 0; k < n_tau; ++k) {\n        int64_t d = (int64_t)d0 + (int64_t)k * step;",
     "    for (int32_t k = 0; k < n_tau - 1; ++k) {\n        int64_t d = (int64_t)d0 + (int64_t)k * step;",
     ["tests/test_oracle_maxdelay_pins.py"], []),
    ("smooth statistic: row centres not shifted by one half", "stt_oracle_ext.c",
     "double u = t, v = f - 0.5;", "double u = t, v = f;", SMOOTH, []),
    ("smooth gradient: start and end time weights transposed", "stt_oracle_ext.c",
     "        gr[0] += (1 - xi) * du;\n        gr[1] += xi * du;", "        gr[0] += xi * du;\n        gr[1] += (1 - xi) * du;",
     SMOOTH, []),
    ("refinement: delay moved against its gradient", "stt_oracle_ext.c",
     "        if (g[5] > 0) th[5] += ems;\n        else if (g[5] < 0) th[5] -= ems;",
     "        if (g[5] > 0) th[5] -= ems;\n        else if (g[5] < 0) th[5] += ems;",
     SMOOTH, []),
    ("refinement: step schedule reversed", "stt_oracle_ext.c",
     "const double epx = sched[0] + w * (sched[1] - sched[0]);", "const double epx = sched[1] + w * (sched[0] - sched[1]);",
     SMOOTH, []),
]


def _build(tmp, sources):
    out = os.path.join(tmp, "libstt_oracle.so")
    srcs = [os.path.join(tmp, s) for s in ("stt_oracle.c", "stt_oracle_ext.c")]
    for s in ("stt_oracle.c", "stt_oracle_ext.c"):
        with open(os.path.join(tmp, s), "w") as fh:
            fh.write(sources[s])
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
                    "-o", out, *srcs, "-lm"], check=True, capture_output=True)
    return out


def _run_pins(lib, files, extra):
    env = dict(os.environ, STT_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        *extra, *files], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-1500:]


def _sources():
    out = {}
    for s in ("stt_oracle.c", "stt_oracle_ext.c"):
        with open(os.path.join(ORACLE, s)) as fh:
            out[s] = fh.read()
    return out


@pytest.fixture(scope="module")
def gcc():
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")


def test_unchanged_copy_passes_the_pins(gcc, tmp_path):
    lib = _build(str(tmp_path), _sources())
    files = sorted({f for m in MUTANTS for f in m[4]})
    rc, log = _run_pins(lib, files, NO_PHILOX)
    assert rc == 0, log


@pytest.mark.parametrize("name,src,old,new,files,extra", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(gcc, tmp_path, name, src, old, new, files, extra):
    srcs = _sources()
    assert srcs[src].count(old) == 1, f"the text to change is not unique in {src}"
    srcs[src] = srcs[src].replace(old, new)
    lib = _build(str(tmp_path), srcs)
    rc, log = _run_pins(lib, files, extra)
    assert rc == 1, f"{name}: the pins did not fail (exit {rc})\n{log}"


# Mistakes in the oracle's Python modules: (name, module file, exact text, replacement, pin file)
PY_MUTANTS = [
    ("FAP counts strictly louder maps only", "significance.py",
     "return key_score(kr) >= key_score(kq)", "return key_score(kr) > key_score(kq)",
     "tests/test_oracle_significance_pins.py"),
    ("threshold at the floor(alpha n)-th map", "significance.py",
     "m = max(1, math.ceil(alpha * len(z)))", "m = max(1, math.floor(alpha * len(z)))",
     "tests/test_oracle_significance_pins.py"),
    ("symmetric instead of periodic Hann window", "mapform.py",
     "return np.sin(np.pi * n / M) ** 2", "return np.sin(np.pi * n / (M - 1)) ** 2",
     "tests/test_oracle_mapform_pins.py"),
    ("conjugate on J instead of I", "mapform.py",
     "np.conj(spec_i) * spec_j[tj]", "spec_i * np.conj(spec_j[tj])", "tests/test_oracle_mapform_pins.py"),
    ("P' averages the half-overlapping neighbours too", "mapform.py",
     "abs(u - t) >= 2 and 0 <= u < T", "abs(u - t) >= 1 and 0 <= u < T", "tests/test_oracle_mapform_pins.py"),
    ("window mean square 1/2 instead of 3/8", "mapform.py",
     "HANN_MEAN_SQUARE = 3.0 / 8.0", "HANN_MEAN_SQUARE = 1.0 / 2.0", "tests/test_oracle_mapform_pins.py"),
    ("patch delay moved the wrong way", "oracle.py",
     'out["dtau"] = out["dtau"].astype(np.int64) + center', 'out["dtau"] = out["dtau"].astype(np.int64) - center',
     "tests/test_oracle_patch_pins.py"),
    ("FP16 scale exponent one too high", "oracle.py",
     "e = (k if fr > 0.5 else k - 1) - 15", "e = (k if fr > 0.5 else k - 1) - 14", "tests/test_oracle_ext_pins.py"),
    ("FP16 phase truncated instead of rounded", "oracle.py",
     "np.rint(turns * 65536.0)", "np.floor(turns * 65536.0)", "tests/test_oracle_ext_pins.py"),
]


def _tree_copy(tmp):
    ign = shutil.ignore_patterns("__pycache__", "*.pyc")
    for d in ("tests", "oracle", "synth"):
        shutil.copytree(os.path.join(ROOT, d), os.path.join(tmp, d), ignore=ign)
    return tmp


def _run_in(tree, pin):
    env = {k: v for k, v in os.environ.items() if k != "STT_ORACLE_LIB"}
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu", pin],
                       cwd=tree, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-1500:]


@pytest.fixture(scope="module")
def built_oracle(gcc):
    import oracle
    if not os.path.exists(os.path.join(ORACLE, "libstt_oracle.so")):
        oracle.build()


def test_unchanged_tree_copy_passes_the_python_pins(built_oracle, tmp_path):
    tree = _tree_copy(str(tmp_path))
    for pin in sorted({m[4] for m in PY_MUTANTS}):
        rc, log = _run_in(tree, pin)
        assert rc == 0, log


@pytest.mark.parametrize("name,mod,old,new,pin", PY_MUTANTS, ids=[m[0] for m in PY_MUTANTS])
def test_planted_mistake_in_python_oracle_is_caught(built_oracle, tmp_path, name, mod, old, new, pin):
    tree = _tree_copy(str(tmp_path))
    path = os.path.join(tree, "oracle", mod)
    with open(path) as fh:
        text = fh.read()
    assert text.count(old) == 1, f"the text to change is not unique in {mod}"
    with open(path, "w") as fh:
        fh.write(text.replace(old, new))
    rc, log = _run_in(tree, pin)
    assert rc == 1, f"{name}: the pins did not fail (exit {rc})\n{log}"
