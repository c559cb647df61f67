"""C-ABI library checks that need no GPU: the shared library loads, exports
every symbol include/h2ulv.h declares, validates arguments before touching the
device, and its host setup (cluster tree, near/far lists; Sec. I, III-D) is
integer-identical to the independent oracle implementation."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import h2ulv_ref as O
from paper_2208_10907_amd import h2ulv as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "h2ulv.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(h2ulv_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol(lib):
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(H.EXPORTS) == syms


def test_params_default(lib):
    p = H.Params()
    assert lib.h2ulv_params_default(C.byref(p)) == 0
    assert p.struct_size == C.sizeof(H.Params)
    assert (p.kernel, p.diag, p.eta, p.leaf_size, p.tol, p.far_sample) == (0, 1e3, 1.0, 256, 1e-8, 32)
    assert (p.sketch_fallback, p.sketch_min_level) == (1, 0)
    assert lib.h2ulv_params_default(None) == H.ERR_INVALID_ARG


def test_invalid_arguments_rejected_before_device_work(lib):
    p = H.make_params(leaf=64)
    out = C.c_void_p()
    assert lib.h2ulv_factorize(None, 10, C.byref(p), None, None, C.byref(out)) == H.ERR_INVALID_ARG
    assert out.value is None
    for field, val in (("leaf_size", 1), ("eta", -1.0), ("tol", float("nan")), ("rank_cap", -1),
                       ("kernel", 9), ("far_sample", -3), ("precision", 5),
                       ("sketch_fallback", 2), ("sketch_min_level", -1)):
        q = H.make_params(leaf=64)
        setattr(q, field, val)
        dummy = C.c_void_p(16)  # never dereferenced: validation fails first
        assert lib.h2ulv_factorize(dummy, 10, C.byref(q), None, None, C.byref(out)) == H.ERR_INVALID_ARG
        assert "must" in lib.h2ulv_last_error().decode() or "unknown" in lib.h2ulv_last_error().decode()
    bad = H.make_params(leaf=64)
    bad.struct_size = 4
    assert lib.h2ulv_factorize(C.c_void_p(16), 10, C.byref(bad), None, None, C.byref(out)) == H.ERR_INVALID_ARG
    # an allocator with a NULL function is refused before any device work
    half = H.Allocator(None, H.ALLOC_FN(lambda c, n, s: None), H.FREE_FN())
    assert lib.h2ulv_factorize(C.c_void_p(16), 10, C.byref(p), C.byref(half), None,
                               C.byref(out)) == H.ERR_INVALID_ARG
    assert lib.h2ulv_solve(None, None, 1, 1, None) == H.ERR_INVALID_ARG
    assert lib.h2ulv_refine(None, None, 1, None, 1, 1, 1e-10, 5, None, None, None) == H.ERR_INVALID_ARG
    assert lib.h2ulv_status_string(H.ERR_SINGULAR) == b"singular block"


def test_structure_rejects_nan_points():
    X = W.cube_points(100, 1)
    X[5, 1] = np.nan
    with pytest.raises(H.H2ULVError) as e:
        H.Structure(X, H.make_params(leaf=16))
    assert e.value.status == H.ERR_INVALID_ARG


@pytest.mark.parametrize("case", [
    ("cube", 2048, 64, 1.0, "kd"), ("cube-ragged", 3001, 64, 1.0, "kd"),
    ("sphere", 5000, 100, 1.0, "kd"), ("line", 64, 16, 1.5, "kd"), ("hss", 1024, 64, 0.0, "kd"),
    ("boxes", 9000, 128, 1.0, "kd"), ("ellipsoids", 6000, 64, 1.0, "kmeans"),
    ("sphere", 5000, 100, 1.0, "kmeans"), ("cube-ragged", 3001, 64, 1.0, "kmeans"),
    ("cube", 2048, 64, 1.0, "kd", "blr2"), ("sphere", 5000, 100, 1.5, "kd", "blr2")])
def test_structure_identical_to_oracle(case):
    name, n, leaf, eta, part = case[:5]
    structure = case[5] if len(case) > 5 else "h2"
    X = {"cube": lambda: W.cube_points(n, 1), "cube-ragged": lambda: W.cube_points(n, 2),
         "sphere": lambda: W.sphere_points(n, 2), "line": lambda: W.line_points(n),
         "hss": lambda: W.cube_points(n, 5), "boxes": lambda: W.box_problem(3)[:n],
         "ellipsoids": lambda: W.ellipsoid_points(n, 7)}[name]()
    s = H.Structure(X, H.make_params(leaf=leaf, eta=eta, partition=part, structure=structure))
    t = O.build_tree(X, leaf, part)
    near, far = (O.build_flat_lists if structure == "blr2" else O.build_lists)(t, eta)
    assert s.L == t.L
    assert np.array_equal(s.perm(), t.perm)
    for lev in range(t.L + 1):
        n2, f2 = s.lists(lev)
        assert n2 == near[lev] and f2 == far[lev]
        c, r = s.geometry(lev)
        assert np.array_equal(c, t.centre[lev]) and np.array_equal(r, t.radius[lev])


def test_build_rejects_kernels_with_scratch():
    """The build fails when any kernel's resource report shows scratch memory
    per lane (register spills, stack arrays); the parser finds exactly those."""
    from paper_2208_10907_amd import build as B
    txt = "\n".join([
        "a.hip:1:1: remark: Function Name: _Zfoo [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     VGPRs: 250 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     ScratchSize [bytes/lane]: 16 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark: Function Name: _Zbar [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
    ])
    assert B.scratch_users(txt) == [("_Zfoo", 16)]
    assert "-Rpass-analysis=kernel-resource-usage" in B.HIP_FLAGS


def test_separate_bases_parameter_checks():
    """The advection kernel needs alpha >= |drift| (decay in every direction);
    separate bases are refused with the flat structure or mixed precision,
    before any device work."""
    X = W.cube_points(200, 1)
    bad = [dict(kernel=H.ADVECTION, alpha=0.5, drift=(0.6, 0.0, 0.0)),
           dict(kernel=H.ADVECTION, alpha=1.0, drift=(float("nan"), 0.0, 0.0)),
           dict(kernel=H.ADVECTION, alpha=1.0, drift=(0.5, 0.0, 0.0), structure="blr2"),
           dict(bases="separate", precision=H.MIXED)]
    for kw in bad:
        with pytest.raises(H.H2ULVError) as e:
            H.Structure(X, H.make_params(leaf=32, **kw))
        assert e.value.status == H.ERR_INVALID_ARG, kw
    with pytest.raises(O.OracleError):
        O.factorize(X, O.Params(kernel=O.ADVECTION, alpha=0.5, drift=(0.6, 0.0, 0.0)))


def test_rankmodel_load_rejects_bad_files_before_device_work(lib, tmp_path):
    """h2ulv_rankmodel_load checks the file (magic, format version, parameter
    count, exact size) before it allocates anything on a device, so every bad
    file is refused here, without a GPU; NULL arguments too."""
    import struct
    out = C.c_void_p(123)
    assert lib.h2ulv_rankmodel_load(str(tmp_path / "missing.h2rm").encode(),
                                    C.byref(out)) == H.ERR_INVALID_ARG
    assert out.value is None
    n = H.MLP_NPARAM
    good_head = b"H2RM" + struct.pack("<IIq", 1, n, 7)
    body = bytes(3 * n * 4)
    cases = {"foreign": b"XXXX" + good_head[4:] + body,
             "version": b"H2RM" + struct.pack("<IIq", 2, n, 7) + body,
             "count": b"H2RM" + struct.pack("<IIq", 1, n - 1, 7) + body,
             "negative step": b"H2RM" + struct.pack("<IIq", 1, n, -1) + body,
             "truncated": good_head + body[:-4],
             "oversized": good_head + body + b"\0",
             "empty": b""}
    for name, data in cases.items():
        f = tmp_path / f"{name}.h2rm"
        f.write_bytes(data)
        out = C.c_void_p(123)
        assert lib.h2ulv_rankmodel_load(str(f).encode(), C.byref(out)) == H.ERR_INVALID_ARG, name
        assert out.value is None, name
        assert lib.h2ulv_last_error().decode(), name
    assert lib.h2ulv_rankmodel_load(None, C.byref(out)) == H.ERR_INVALID_ARG
    assert lib.h2ulv_rankmodel_load(str(tmp_path / "x").encode(), None) == H.ERR_INVALID_ARG
    assert lib.h2ulv_rankmodel_save(None, str(tmp_path / "x").encode()) == H.ERR_INVALID_ARG
