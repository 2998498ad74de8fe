"""CPU checks of the C-ABI library: it loads, exports exactly what
include/frsvt.h declares, and rejects invalid arguments before touching the
device (no GPU is needed for these)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "frsvt.h")
LIB = os.path.join(ROOT, "paper_1509_00296_amd", "libfrsvt.so")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"FRSVT_API\s+[\w\s\*]+?\b(\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1509_00296_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_paper_calls():
    names = _declared()
    for required in ("svt", "frsvt", "wsvt", "rpca_ialm", "wsvt_batched", "frsvt_create",
                     "frsvt_destroy"):
        assert required in names


def test_exports_match_header(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = sorted({line.split()[-1] for line in out.splitlines() if " T " in line})
    assert exported == _declared()
    for name in _declared():
        assert hasattr(lib, name)


def test_status_strings(lib):
    lib.frsvt_status_string.restype = ctypes.c_char_p
    assert lib.frsvt_status_string(0) == b"success"
    assert b"argument" in lib.frsvt_status_string(-3)
    assert b"non-finite" in lib.frsvt_status_string(-102)


def test_null_handle_rejected(lib):
    assert lib.svt(None, 0, 10, 10, None, 10, ctypes.c_double(1.0), None, 10, None) == -1
    assert lib.frsvt_destroy(None) == -1


def test_argument_validation_precedes_device_use(lib):
    # A dummy, never-dereferenced handle: every call below has an invalid
    # argument, which the library reports before it touches the handle.
    dummy = ctypes.c_void_p(ctypes.addressof(ctypes.create_string_buffer(64)))
    buf = ctypes.c_void_p(ctypes.addressof(ctypes.create_string_buffer(64)))
    d = ctypes.c_double
    lib.svt.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                        ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p,
                        ctypes.c_int64, ctypes.c_void_p]
    assert lib.svt(dummy, 7, 10, 10, buf, 10, 1.0, buf, 10, None) == -2      # precision
    assert lib.svt(dummy, 0, 0, 10, buf, 10, 1.0, buf, 10, None) == -3       # m < 1
    assert lib.svt(dummy, 0, 10, 0, buf, 10, 1.0, buf, 10, None) == -4       # n < 1
    assert lib.svt(dummy, 0, 10, 10, None, 10, 1.0, buf, 10, None) == -5     # A NULL
    assert lib.svt(dummy, 0, 10, 10, buf, 9, 1.0, buf, 10, None) == -6       # lda < m
    assert lib.svt(dummy, 0, 10, 10, buf, 10, -1.0, buf, 10, None) == -7     # tau < 0
    assert lib.svt(dummy, 0, 10, 10, buf, 10, float("nan"), buf, 10, None) == -7
    assert lib.svt(dummy, 0, 10, 10, buf, 10, 1.0, None, 10, None) == -8     # X NULL
    assert lib.svt(dummy, 0, 10, 10, buf, 10, 1.0, buf, 5, None) == -9       # ldx < m
    i32, i64, u64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
    lib.frsvt.argtypes = [vp, ctypes.c_int, i64, i64, vp, i64, d, i32, i32, i32, vp, i32, i64,
                          u64, u64, vp, i64, vp, i64, vp]
    args = [dummy, 0, 20, 30, buf, 20, 1.0, 5, 3, 1, None, 0, 20, 0, 0, buf, 20, None, 20, None]

    def call(**kw):
        a = list(args)
        names = ["h", "prec", "m", "n", "A", "lda", "tau", "k", "p", "q", "Qp", "rp", "ldqp",
                 "seed", "ctr", "X", "ldx", "Qo", "ldqo", "r"]
        for key, val in kw.items():
            a[names.index(key)] = val
        return lib.frsvt(*a)
    assert call(k=0, p=0) == -8
    assert call(p=-1) == -9
    assert call(q=-1) == -10
    assert call(Qp=buf, rp=21) == -12          # r_prev > min(m, n)
    assert call(Qp=buf, rp=3, ldqp=10) == -13  # ldq_prev < min(m, n)
    assert call(X=None) == -16
    assert call(ldx=10) == -17
    assert call(Qo=buf, ldqo=5) == -19
    lib.wsvt.argtypes = [vp, ctypes.c_int, i64, i64, vp, i64, vp, vp, i64, vp]
    assert lib.wsvt(dummy, 0, 10, 10, buf, 10, None, buf, 10, None) == -7   # w NULL
    lib.rpca_ialm.argtypes = [vp, ctypes.c_int, i64, i64, vp, i64, d, vp, vp, i64, vp, i64, vp]
    assert lib.rpca_ialm(dummy, 0, 10, 10, buf, 10, 0.0, None, buf, 10, buf, 10, None) == -7
    assert lib.rpca_ialm(dummy, 0, 10, 10, buf, 10, 0.1, None, None, 10, buf, 10, None) == -9
    import paper_1509_00296_amd as fr
    for field, val in (("ap_gamma", 1.5), ("ap", 1), ("keep", -1), ("r_init", 11), ("r_init", 2)):
        op = fr.RpcaOpts()
        lib.frsvt_rpca_default_opts(ctypes.byref(op))
        setattr(op, field, val)
        if field == "ap":
            op.ap_a = 0                       # a >= 1 required
        if field == "ap_gamma":
            op.ap = 1
        # r_init = 11 > min(m, n); r_init = 2 without q_init
        assert lib.rpca_ialm(dummy, 0, 10, 10, buf, 10, 0.1, ctypes.byref(op), buf, 10, buf, 10,
                             None) == -8, field
    lib.tensor_rpca.argtypes = [vp, ctypes.c_int, i64, i64, i64, vp, vp, d, vp, vp, vp, vp]
    al = (d * 3)(0.2, 0.3, 0.5)
    bad_al = (d * 3)(0.2, -0.3, 0.5)
    assert lib.tensor_rpca(dummy, 0, 4, 0, 5, buf, al, 0.1, None, buf, buf, None) == -4     # I2 < 1
    assert lib.tensor_rpca(dummy, 0, 4, 3, 5, buf, None, 0.1, None, buf, buf, None) == -7   # alpha NULL
    assert lib.tensor_rpca(dummy, 0, 4, 3, 5, buf, bad_al, 0.1, None, buf, buf, None) == -7
    assert lib.tensor_rpca(dummy, 0, 4, 3, 5, buf, al, 0.0, None, buf, buf, None) == -8     # lambda
    top = fr.TensorOpts()
    lib.frsvt_tensor_default_opts(ctypes.byref(top))
    top.rho = 0.5
    assert lib.tensor_rpca(dummy, 0, 4, 3, 5, buf, al, 0.1, ctypes.byref(top), buf, buf, None) == -9
    buf2 = ctypes.c_void_p(ctypes.addressof(ctypes.create_string_buffer(64)))
    assert lib.tensor_rpca(dummy, 0, 4, 3, 5, buf, al, 0.1, None, buf2, buf2, None) == -11  # L aliases E
    lib.wsvt_batched.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp]
    assert lib.wsvt_batched(dummy, -1, None, None, None, None, None, None, None) == -2


def test_create_without_gpu_fails_cleanly(lib):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    h = ctypes.c_void_p()
    rc = lib.frsvt_create(ctypes.byref(h), 0, None)
    assert rc in (-100, -104, -2)
    assert not h.value


def test_binding_refuses_missing_library(tmp_path):
    import paper_1509_00296_amd as fr
    with pytest.raises(ImportError):
        fr.library(str(tmp_path / "missing.so"))


def test_struct_layouts_match_header(tmp_path):
    """The Python binding's ctypes structures have the sizes and field
    offsets that a C compiler gives the header's structures."""
    import paper_1509_00296_amd as fr
    src = tmp_path / "sizes.c"
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "frsvt.h"\n'
        "int main(void) {\n"
        '  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(frsvt_rpca_opts), sizeof(frsvt_rpca_stats),\n'
        "         offsetof(frsvt_rpca_opts, seed), offsetof(frsvt_rpca_opts, q_final),\n"
        "         offsetof(frsvt_rpca_stats, resid_est), sizeof(frsvt_wsvt_rule));\n"
        '  printf("%zu %zu %zu\\n", sizeof(frsvt_lrr_opts), sizeof(frsvt_lrr_stats),\n'
        "         offsetof(frsvt_lrr_opts, seed));\n"
        '  printf("%zu %zu %zu %zu\\n", sizeof(frsvt_tensor_opts), sizeof(frsvt_tensor_stats),\n'
        "         offsetof(frsvt_tensor_opts, seed), offsetof(frsvt_tensor_stats, resid));\n"
        "  return 0;\n}\n")
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [ctypes.sizeof(fr.RpcaOpts), ctypes.sizeof(fr.RpcaStats), fr.RpcaOpts.seed.offset,
            fr.RpcaOpts.q_final.offset, fr.RpcaStats.resid_est.offset, ctypes.sizeof(fr.WsvtRule),
            ctypes.sizeof(fr.LrrOpts), ctypes.sizeof(fr.LrrStats), fr.LrrOpts.seed.offset,
            ctypes.sizeof(fr.TensorOpts), ctypes.sizeof(fr.TensorStats), fr.TensorOpts.seed.offset,
            fr.TensorStats.resid.offset]
    assert got == want
