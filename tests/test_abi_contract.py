"""Host-side contract of the C ABI: the library loads, exports every function the
public header declares, and rejects bad arguments before touching a device.
No GPU is needed (no compute call is made)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1808_07284_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("library not built")
    return L, L.load()


def declared_functions():
    names = []
    inc = os.path.join(ROOT, "include")
    for fn in sorted(os.listdir(inc)):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(emd_\w+)\s*\(", text, flags=re.M)
    return names


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("emd_decompose", "emd_pdhg_solve", "emd_adjoint_source", "emd_plan_create"):
        assert n in names


def test_every_declared_symbol_is_exported():
    L, lib = _lib()
    names = declared_functions()
    assert set(names) == set(L.EXPORTED)
    for n in names:
        assert hasattr(lib, n), n


def test_params_default_are_the_papers():
    L, lib = _lib()
    p = L.Params()
    assert lib.emd_params_default(C.byref(p)) == 0
    assert (p.eps, p.xi, p.zeta, p.delta) == (1e-4, 0.5, 0.99, 1e5)
    assert p.ls_mode == L.LS_L2 and p.mass_mode == L.MASS_BALANCE and p.precision == L.F32
    assert lib.emd_params_default(None) == 2


def _create(L, lib, descs, batch_len, **over):
    p = L.Params()
    lib.emd_params_default(C.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    arr = (L.GatherDesc * max(len(descs), 1))()
    for k, d in enumerate(descs):
        arr[k] = L.GatherDesc(*d)
    h = C.c_void_p()
    st = lib.emd_plan_create(arr, len(descs), batch_len, C.byref(p), C.byref(h))
    if st == 0:
        lib.emd_plan_destroy(h)
    return st, lib.emd_last_error().decode()


@pytest.mark.parametrize("descs,batch,over,code", [
    ([], 10, {}, 1),                                        # no gathers
    ([(0, 5, 1.0, 1.0, 0)], 10, {}, 1),                     # nr = 0
    ([(2, 5, 0.0, 1.0, 0)], 10, {}, 1),                     # dx = 0
    ([(2, 5, 1.0, float("nan"), 0)], 10, {}, 1),            # dt NaN
    ([(2, 5, 1.0, 1.0, 1)], 10, {}, 1),                     # past the batch end
    ([(2, 5, 1.0, 1.0, 0), (1, 5, 1.0, 1.0, 8)], 20, {}, 1),  # overlapping gathers
    ([(2, 5, 1.0, 1.0, 0)], 10, {"xi": 1.0}, 1),
    ([(2, 5, 1.0, 1.0, 0)], 10, {"zeta": 0.0}, 1),
    ([(2, 5, 1.0, 1.0, 0)], 10, {"delta": -1.0}, 1),
    ([(2, 5, 1.0, 1.0, 0)], 10, {"max_iter": 0}, 1),
    ([(2, 5, 1.0, 1.0, 0)], 10, {"check_every": 0}, 1),
    ([(2, 5, 1.0, 1.0, 0)], 10, {"precision": 7}, 1),
    ([(2, 5, 1.0, 1.0, 0)], 10, {"mass_mode": 3}, 1),
    ([(2, 5, 1.0, 1.0, 0)], 10, {"sweeps_per_sync": 1}, 1),
    ([(2, 5, 1.0, 1.0, 0)], 10, {"sweeps_per_sync": 3}, 1),  # chunks hold whole sweep pairs
    ([(2, 5, 1.0, 1.0, 0)], 10, {"sweeps_per_sync": -2}, 1),
    ([(2, 5, 1.0, 1.0, 0)], 10, {"iters_per_sweep": 4, "ls_mode": 2}, 1),
    ([(2, 5, 1.0, 1.0, 0)], 10, {"iters_per_sweep": 2}, 1),                       # needs fixed steps
    ([(2, 5, 1.0, 1.0, 0)], 10, {"iters_per_sweep": 3}, 1),                       # needs fixed steps
    ([(2, 5, 1.0, 1.0, 0)], 10, {"iters_per_sweep": 2, "ls_mode": 2, "check_every": 5}, 1),  # odd checks
    ([(2, 5, 1.0, 1.0, 0)], 10, {"iters_per_sweep": 3, "ls_mode": 2, "check_every": 10}, 1),  # not x3
    ([(2, 5, 1.0, 1.0, 0)], 10, {"iters_per_sweep": 3, "ls_mode": 2, "check_every": 12, "precision": 1}, 1),
    ([(2, 5, 1.0, 1.0, 0)], 10, {"sweeps_per_sync": 4098}, 1),
    ([(2, 5, 1.0, 1.0, 0)], 10, {"ls_mode": 3}, 1),         # unknown linesearch test
    # a field region of a gather (nr rows of nt rounded up to 32) may not pass 1 GiB
    ([(16384, 16385, 1.0, 1.0, 0)], 16384 * 16385, {}, 1),
    ([(8192, 16385, 1.0, 1.0, 0)], 8192 * 16385, {"precision": 1}, 1),
    ([(1, 1 << 31, 1.0, 1.0, 0)], 1 << 31, {}, 1),          # one trace of 2^31 samples: 8 GiB
    ([(2, 5, 1.0, 1.0, 0)], 10, {"max_ls_trials": -1}, 1),
])
def test_plan_create_rejects_bad_arguments(descs, batch, over, code):
    L, lib = _lib()
    st, msg = _create(L, lib, descs, batch, **over)
    assert st == code, msg
    assert msg


def test_plan_create_without_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L, lib = _lib()
    st, msg = _create(L, lib, [(2, 5, 1.0, 1.0, 0)], 10)
    assert st == 3, msg


@pytest.mark.parametrize("desc,precision", [((16384, 16384, 1.0, 1.0, 0), 0), ((8192, 16384, 1.0, 1.0, 0), 1)])
def test_field_regions_of_exactly_1_gib_pass_validation(desc, precision):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present (the GPU tests cover this size)")
    L, lib = _lib()
    st, msg = _create(L, lib, [desc], desc[0] * desc[1], precision=precision)
    assert st == 3, msg  # past validation, then: no device on this host


def test_null_pointers_are_rejected():
    L, lib = _lib()
    assert lib.emd_decompose(None, None, None, None, None, None, None, None) == 2
    assert lib.emd_pdhg_solve(None, None, None, None, 0, None, None, None, None) == 2
    assert lib.emd_adjoint_source(None, None, None, None, None, None, None, None) == 2
    assert lib.emd_plan_set_history(None, None, 0) == 2
    assert lib.emd_plan_destroy(None) == 0
    assert lib.emd_status_string(1) == b"EMD_ERR_INVALID_ARGUMENT"


def test_noalloc_decompose_rejects_bad_arguments():
    # every case fails validation on the host, before any device call (the pointers
    # are never dereferenced); skipped where a GPU could be reached by mistake
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L, lib = _lib()
    D = L.GatherDesc
    p = [C.c_void_p(0x1000 * (k + 1)) for k in range(4)]

    def call(descs, n, precision=0, mode=0, ptrs=p):
        arr = (D * len(descs))(*descs)
        return lib.emd_decompose_noalloc(arr, n, precision, mode, ptrs[0], ptrs[1], ptrs[2], None, None,
                                         ptrs[3], None), lib.emd_last_error()

    one = [D(4, 8, 0.1, 0.1, 0)]
    assert call(one, 1, ptrs=[None, p[1], p[2], p[3]])[0] == 2
    assert call(one, 1, ptrs=[p[0], p[1], p[0], p[3]])[0] == 1            # s_out aliases pcal
    st, msg = call([D(1, 4, 1.0, 1.0, 4 * k) for k in range(65)], 65)
    assert st == 1 and b"static scratch" in msg
    assert call(one, 0)[0] == 1
    assert call(one, 1, precision=2)[0] == 1
    assert call(one, 1, mode=3)[0] == 1
    assert call([D(0, 8, 0.1, 0.1, 0)], 1)[0] == 1
    assert call([D(4, 8, 0.0, 0.1, 0)], 1)[0] == 1
    assert call([D(4, 8, 0.1, 0.1, -1)], 1)[0] == 1
    assert call([D(2, 4, 1.0, 1.0, 0), D(2, 4, 1.0, 1.0, 4)], 2)[0] == 1  # overlap
    st, _ = call(one, 1)                                                   # valid: no device here
    assert st in (3, 4)


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1808_07284_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "emd_oracle" not in text and "liboracle" not in text, fn


def _header_structs():
    text = open(os.path.join(ROOT, "include", "emd_mi355x.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef\s+struct\s*\{(.*?)\}\s*(emd_\w+)\s*;", text, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            ctype, names = decl.split(None, 1)
            fields += [(n.strip(), ctype) for n in names.split(",")]
        out[name] = fields
    return out


def test_binding_structs_mirror_the_header():
    from paper_1808_07284_amd import _lib as L
    ctypes_of = {"int32_t": C.c_int32, "int64_t": C.c_int64, "double": C.c_double}
    structs = _header_structs()
    pairs = {"emd_gather_desc": L.GatherDesc, "emd_params": L.Params,
             "emd_solve_info": L.SolveInfo, "emd_plan_stats": L.PlanStats,
             "emd_gather_state": L.GatherState}
    assert set(pairs) <= set(structs)
    for hname, cls in pairs.items():
        assert [(n, ctypes_of[t]) for n, t in structs[hname]] == \
            [(n, t) for n, t in cls._fields_], hname


def test_autotune_cache_key():
    from paper_1808_07284_amd.api import autotune_key
    from paper_1808_07284_amd import F32, F64
    k = autotune_key("gfx950", "7.0", F32, [(300, 2000), (200, 1500)])
    from paper_1808_07284_amd.api import AUTOTUNE_REVISION
    assert k.startswith("gfx950|rocm 7.0|f32|2 gathers|")
    assert k.endswith(f"|tuner {AUTOTUNE_REVISION}")
    assert k == autotune_key("gfx950", "7.0", F32, [(300, 2000), (200, 1500)])
    # order, sizes, precision, architecture and ROCm version all separate entries
    others = [autotune_key("gfx950", "7.0", F32, [(200, 1500), (300, 2000)]),
              autotune_key("gfx950", "7.0", F32, [(300, 2000), (200, 1501)]),
              autotune_key("gfx950", "7.0", F64, [(300, 2000), (200, 1500)]),
              autotune_key("gfx942", "7.0", F32, [(300, 2000), (200, 1500)]),
              autotune_key("gfx950", "7.2", F32, [(300, 2000), (200, 1500)])]
    assert k not in others and len(set(others)) == len(others)
