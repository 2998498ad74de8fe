"""Plant plausible mistakes in copies of the oracle source (on the CPU) and
check that the oracle's pin tests reject every one of them."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "frsvt_oracle.c")
PIN_FILES = ["tests/test_oracle_rng.py", "tests/test_oracle_linalg.py",
             "tests/test_oracle_svt.py", "tests/test_oracle_frsvt.py",
             "tests/test_oracle_rpca_grad.py", "tests/test_oracle_ap.py", "tests/test_oracle_lrr.py",
             "tests/test_oracle_resid_check.py"]

# (name, original text, planted mistake[, the pin file that should reject it
# first: run ahead of the others so that the -x run stops early])
MUTANTS = [
    ("philox_multiplier", "0xD2511F53u * (uint64_t)c0", "0xD2511F55u * (uint64_t)c0"),
    ("philox_key_bump", "k1 += 0xBB67AE85u;", "k1 += 0xBB67AE84u;"),
    ("uniform_bits", "double lo = (double)(b >> 6);", "double lo = (double)(b >> 7);"),
    ("box_muller_radius", "sqrt(-2.0 * log(u1))", "sqrt(-1.0 * log(u1))"),
    ("householder_beta_sign", "*beta = -v0 / alpha;", "*beta = v0 / alpha;"),
    ("qrcp_no_pivot", "if (nc > best_norm) {", "if (nc > best_norm && c == j) {"),
    ("jacobi_rotation_sign", "gq[i] = s * a + c * b;", "gq[i] = -s * a + c * b;"),
    ("jacobi_v_not_rotated", "vq[i] = s * a + c * b;", "vq[i] = b;"),
    ("soft_threshold_half", "double a = fabs(x) - tau;", "double a = fabs(x) - 0.5 * tau;"),
    ("frsvt_swapped_factors", "mat_mul(nh, s, s, H, nh, UC, s, HWV, nh);",
     "mat_mul(nh, s, s, H, nh, VC, s, HWV, nh);"),
    ("frsvt_one_power_step_short", "for (int it = 0; it < q; ++it) {",
     "for (int it = 1; it < q; ++it) {"),
    ("rp_no_partial_orthogonalisation", "for (int pass = 0; pass < 2; ++pass)\n            for (int64_t c = 0; c < have + j; ++c) {",
     "for (int pass = 0; pass < 0; ++pass)\n            for (int64_t c = 0; c < have + j; ++c) {"),
    ("frsvt_rank_off_by_one", "shr[i] = i < keep ? D[i] : soft_shrink(D[i], tau);\n        if (shr[i] > 0.0) ++r;",
     "shr[i] = i < keep ? D[i] : soft_shrink(D[i], tau);\n        if (shr[i] > 0.0 && i > 0) ++r;"),
    ("frsvt_partial_ignored", "shr[i] = i < keep ? D[i] : soft_shrink(D[i], tau);",
     "shr[i] = soft_shrink(D[i], tau);"),
    ("psvt_keep_off_by_one", "shr[i] = i < keep ? S[i] : soft_shrink(S[i], tau);",
     "shr[i] = i <= keep ? S[i] : soft_shrink(S[i], tau);"),
    ("ap_branch_swapped", "const int64_t pn = r_prev < l_prev ? ap_a : (int64_t)ceil(ap_rho * (double)mh);",
     "const int64_t pn = r_prev <= l_prev ? ap_a : (int64_t)ceil(ap_rho * (double)mh);"),
    ("lrr_dual_sign", "Y2[i] += mu * z;", "Y2[i] -= mu * z;"),
    ("lrr_shrink_threshold", "const double thr = lambda / mu;", "const double thr = lambda * mu;"),
    ("lrr_rhs_without_multiplier", "R[i] += J[i] - Y2[i] / mu;", "R[i] += J[i];"),
    ("residual_one_pass", "    for (int pass = 0; pass < 2; ++pass)\n        for (int64_t c = 0; c < r; ++c) {",
     "    for (int pass = 0; pass < 2; ++pass)\n        for (int64_t c = 0; c < r - 1; ++c) {"),
    ("check_keeps_one_less", "            kept = j + 1;\n            break;", "            kept = j;\n            break;",
     "tests/test_oracle_resid_check.py"),
    ("check_basis_not_extended", "AT(B, mh, i, k) = y[i] / nrm;\n            ++k;",
     "AT(B, mh, i, k) = y[i] / nrm;", "tests/test_oracle_resid_check.py"),
    ("check_threshold_squared", "if (est <= tau) {", "if (est <= tau * tau) {",
     "tests/test_oracle_resid_check.py"),
    ("ialm_dual_sign", "AT(Y, m, i, j) += mu * z;", "AT(Y, m, i, j) -= mu * z;"),
    ("ialm_shrink_lambda", "lambda / mu);", "lambda * mu);"),
    ("vjp_antisymmetric_term", "(f[i] + f[j]) / (sg[i] + sg[j])", "(f[i] - f[j]) / (sg[i] + sg[j])"),
    ("vjp_missing_complement", "AT(UPb, m, i, j) + AT(T, m, i, j) - AT(M2, m, i, j);",
     "AT(UPb, m, i, j);"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,orig,bad,first", [m if len(m) == 4 else (*m, None) for m in MUTANTS],
                         ids=[m[0] for m in MUTANTS])
def test_pins_reject_planted_mistake(tmp_path, name, orig, bad, first):
    src = open(SRC).read()
    assert src.count(orig) == 1, f"mutation anchor for {name} not unique"
    mutated = tmp_path / "frsvt_oracle.c"
    mutated.write_text(src.replace(orig, bad))
    (tmp_path / "frsvt_oracle.h").write_text(open(SRC[:-2] + ".h").read())
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(lib),
                           str(mutated), "-lm"])
    env = dict(os.environ, FRSVT_ORACLE_LIB=str(lib))
    proc = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           "--timeout", "120", *([first] if first else []),
                           *[f for f in PIN_FILES if f != first]], cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=900)
    assert proc.returncode != 0, f"mutant {name} survived the pin tests:\n{proc.stdout[-2000:]}"


# The tensor host of the oracle is numpy glue in oracle/__init__.py: its
# mutants are planted in a copy of the package and checked against its pins.
PY_SRC = os.path.join(ROOT, "oracle", "__init__.py")
PY_PIN_FILES = ["tests/test_oracle_tensor.py"]
PY_MUTANTS = [
    ("tensor_shrink_threshold", "shrink(V, lam / (3.0 * mu))", "shrink(V, lam / mu)"),
    ("tensor_svt_ignores_weight", "X, r = svt(M, alpha[i] / mu)", "X, r = svt(M, 1.0 / mu)"),
    ("tensor_dual_sign", "Y[i] = Y[i] + mu * Z", "Y[i] = Y[i] - mu * Z"),
    ("tensor_mean_divisor", "for i in range(3)) / 3.0", "for i in range(3)) / 2.0"),
    ("tensor_input_without_multiplier", "M = unfold(O - E + Y[i] / mu, i)", "M = unfold(O - E, i)"),
    ("tensor_residual_min", "res = max(res, np.linalg.norm(Z) / normO)", "res = min(res, np.linalg.norm(Z) / normO)"),
    ("unfold_row_major_columns", 'reshape(T.shape[mode], -1, order="F")', 'reshape(T.shape[mode], -1, order="C")'),
    ("fold_wrong_axis", "np.moveaxis(T, 0, mode)", "np.moveaxis(T, mode, 0)"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,orig,bad", PY_MUTANTS, ids=[m[0] for m in PY_MUTANTS])
def test_tensor_pins_reject_planted_mistake(tmp_path, name, orig, bad):
    import shutil
    src = open(PY_SRC).read()
    assert src.count(orig) == 1, f"mutation anchor for {name} not unique"
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    for f in ("frsvt_oracle.c", "frsvt_oracle.h", "liboracle.so"):
        if os.path.exists(os.path.join(ROOT, "oracle", f)):
            shutil.copy(os.path.join(ROOT, "oracle", f), pkg / f)
    (pkg / "__init__.py").write_text(src.replace(orig, bad))
    # run from the copy's parent so that `import oracle` finds the mutant first
    env = dict(os.environ, PYTHONPATH=ROOT)
    env.pop("FRSVT_ORACLE_LIB", None)
    proc = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           "--timeout", "120", "--rootdir", ROOT,
                           *[os.path.join(ROOT, f) for f in PY_PIN_FILES]],
                          cwd=str(tmp_path), env=env, capture_output=True, text=True, timeout=900)
    assert proc.returncode != 0, f"mutant {name} survived the pin tests:\n{proc.stdout[-2000:]}"


def test_tensor_mutant_harness_uses_the_copy(tmp_path):
    """The harness above really imports the copy: an unchanged copy passes
    and a copy whose tensor host raises fails."""
    import shutil
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    for f in ("frsvt_oracle.c", "frsvt_oracle.h", "liboracle.so"):
        if os.path.exists(os.path.join(ROOT, "oracle", f)):
            shutil.copy(os.path.join(ROOT, "oracle", f), pkg / f)
    src = open(PY_SRC).read()
    env = dict(os.environ, PYTHONPATH=ROOT)
    env.pop("FRSVT_ORACLE_LIB", None)
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "--rootdir", ROOT,
           os.path.join(ROOT, "tests", "test_oracle_tensor.py")]
    (pkg / "__init__.py").write_text(src)
    assert subprocess.run(cmd, cwd=str(tmp_path), env=env, capture_output=True).returncode == 0
    anchor = "    O = np.asfortranarray(np.asarray(O, dtype=np.float64))\n    shape = O.shape\n"
    assert src.count(anchor) == 1
    (pkg / "__init__.py").write_text(src.replace(anchor, anchor + "    raise RuntimeError('copy')\n"))
    assert subprocess.run(cmd, cwd=str(tmp_path), env=env, capture_output=True).returncode != 0
