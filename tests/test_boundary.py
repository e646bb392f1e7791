"""CPU-side checks of the C-ABI boundary: the library loads and exports every
symbol the header declares, with matching Python declarations.  No GPU call."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rwtrsv.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rwt_[a-z_A-Z0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2609_40159_amd import _lib, build
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    return _lib.load()


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ["rwt_validate", "rwt_analyze", "rwt_rewrite_symbolic", "rwt_rewrite_numeric",
                 "rwt_plan_create", "rwt_solve", "rwt_solve_transpose", "rwt_apply_MT",
                 "rwt_grad_vals"]:
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    import subprocess
    from paper_2609_40159_amd import _lib
    out = subprocess.check_output(["nm", "-D", "--defined-only", _lib.LIB_PATH]).decode()
    exported = set(re.findall(r"\bT (rwt_\w+)", out))
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing
    for s in declared_symbols():
        assert hasattr(lib, s)


def test_python_declarations_cover_header():
    from paper_2609_40159_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared_symbols()


def test_host_only_calls(lib):
    import ctypes as C
    from paper_2609_40159_amd import _lib
    assert lib.rwt_version().startswith(b"rwtrsv")
    assert lib.rwt_validate_ws() >= 16
    # argument errors are reported without touching the device
    sz = C.c_size_t(0)
    assert lib.rwt_analyze_ws(None, C.byref(sz)) == -1
    assert b"NULL" in lib.rwt_last_error_string()
    assert lib.rwt_apply_MT_ws(-1, 0, C.byref(sz)) == -1
    c = _lib.Csr()
    c.n, c.nnz, c.dt = 10, 5, 0
    c.rowptr = 1
    c.colidx = 1
    assert lib.rwt_analyze_ws(C.byref(c), C.byref(sz)) == -4     # nnz < n: diagonal missing
    c.nnz = 1 << 31
    assert lib.rwt_analyze_ws(C.byref(c), C.byref(sz)) == -8
    c.nnz = 30
    assert lib.rwt_analyze_ws(C.byref(c), C.byref(sz)) == 0 and sz.value > 0
    o = _lib.PlanOpts()
    o.algo, o.kmax, o.lanes_per_row = 0, 1, 3
    c.vals = 1
    assert lib.rwt_plan_ws(C.byref(c), C.byref(o), C.byref(sz)) == -1   # lanes not a power of 2
    o.lanes_per_row = 0
    assert lib.rwt_plan_ws(C.byref(c), C.byref(o), C.byref(sz)) == 0
    assert lib.rwt_generate_ws(10, 11, 1, C.byref(sz)) == -1      # more levels than rows
    assert lib.rwt_generate_ws(10, 3, 4, C.byref(sz)) == 0 and sz.value > 0
    assert lib.rwt_gen_rowsets_ws(1 << 16, 1 << 16, C.byref(sz)) == -8
    assert lib.rwt_gen_rowsets_ws(4, 100, C.byref(sz)) == 0 and sz.value > 0
    # environment: sizes, a workspace too small, invalid parameters
    assert lib.rwt_env_ws(10, 11, 1, 5, C.byref(sz)) == -1        # more levels than rows
    assert lib.rwt_env_ws(10, 3, 0, 5, C.byref(sz)) == -1         # no environment
    assert lib.rwt_env_ws(10, 3, 4, 0, C.byref(sz)) == -1         # no move capacity
    assert lib.rwt_env_ws(10, 3, 4, 6, C.byref(sz)) == 0 and sz.value > 0
    need = sz.value
    assert lib.rwt_env_reset(10, 3, 4, 6, None, C.c_void_p(1), need - 1, None) == -7
    assert lib.rwt_env_step(10, 3, 4, 6, None, None, None, None, None, C.c_void_p(1), need,
                            None) == -1
    ep = _lib.EnvParams(1.0, 0.02, 1.0, 1e-6, 1.0, 8, 5, 2, 0, 0, 8)   # decay must be < 1
    c.n = 10
    assert lib.rwt_env_init(C.byref(c), C.c_void_p(1), C.c_void_p(1), C.c_void_p(1),
                            C.c_void_p(1), 3, 4, 6, C.byref(ep), C.c_void_p(1), need, None) == -1
    assert b"parameters" in lib.rwt_last_error_string()
    for field, bad in (("block_rows", (1 << 20) + 1), ("rhs_chunk", 5), ("tune_cols", -1),
                       ("stage_outside", 3)):
        setattr(o, field, bad)
        assert lib.rwt_plan_ws(C.byref(c), C.byref(o), C.byref(sz)) == -1, field
        setattr(o, field, 0)


def test_package_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2609_40159_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError, match="no fallback"):
        _lib.load()


def test_oracle_and_gpu_path_are_independent():
    """Neither side imports the other; the shared input module imports neither."""
    import synth
    ssrc = open(synth.__file__).read()
    assert "oracle" not in ssrc.split('"""', 2)[2] and "paper_2609_40159_amd" not in ssrc
    odir = os.path.join(ROOT, "oracle")
    for f in os.listdir(odir):
        if f.endswith((".py", ".c", ".h")):
            assert "paper_2609_40159_amd" not in open(os.path.join(odir, f)).read(), f
            assert "rwtrsv" not in open(os.path.join(odir, f)).read(), f
    pdir = os.path.join(ROOT, "paper_2609_40159_amd")
    for dirpath, _, files in os.walk(pdir):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "oracle.c" not in txt and "orc_" not in txt, f


def test_struct_layouts_match_header(tmp_path):
    """Every structure the Python binding declares has the size and field
    offsets of its C definition in include/rwtrsv.h (compiled as C99)."""
    import ctypes as C
    import shutil
    import subprocess
    from paper_2609_40159_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    pairs = {"Csr": "rwt_csr", "LevelStats": "rwt_level_stats", "PlanOpts": "rwt_plan_opts",
             "PlanInfo": "rwt_plan_info", "GenParams": "rwt_gen_params",
             "GenResult": "rwt_gen_result", "EnvParams": "rwt_env_params",
             "EnvResult": "rwt_env_result", "BatchMatrix": "rwt_batch_matrix",
             "BatchDesc": "rwt_batch_desc", "CandStats": "rwt_cand_stats",
             "BatchInfo": "rwt_batch_info"}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rwtrsv.h"', 'int main(void) {']
    want = []
    for py, c in pairs.items():
        st = getattr(_lib, py)
        lines.append(f'    printf("%zu\\n", sizeof({c}));')
        want.append(C.sizeof(st))
        for f, _ in st._fields_:
            lines.append(f'    printf("%zu\\n", offsetof({c}, {f}));')
            want.append(getattr(st, f).offset)
    lines += ['    return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I", inc, str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert got == want


def test_python_signatures_match_header_prototypes():
    """Each ctypes declaration has the argument count of the C prototype,
    pointer arguments where the prototype has pointers, and the right
    return kind (status int, size_t, double pointer...)."""
    import ctypes as C
    from paper_2609_40159_amd import _lib
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    protos = dict()
    for m in re.finditer(r"\b([A-Za-z_][\w ]*?\**)\s*\b(rwt_\w+)\s*\(([^;{]*?)\)\s*;", text):
        ret, name, args = m.group(1).strip(), m.group(2), m.group(3).strip()
        params = [] if args in ("", "void") else [a.strip() for a in args.split(",")]
        protos[name] = (ret, params)
    assert sorted(protos) == sorted(_lib.SIGNATURES)
    for name, (restype, argtypes) in _lib.SIGNATURES.items():
        ret, params = protos[name]
        assert len(params) == len(argtypes), (name, params, argtypes)
        for p, t in zip(params, argtypes):
            is_ptr = "*" in p or p.split()[0] in ("rwt_stream_t",)
            ctypes_ptr = t is C.c_void_p or t is C.c_char_p or isinstance(t, type(C.POINTER(C.c_int)))
            assert is_ptr == bool(ctypes_ptr), (name, p, t)
        if ret == "rwt_status":
            assert restype is C.c_int, name
        elif ret == "size_t":
            assert restype is C.c_size_t, name


def test_plan_options_are_checked_by_name(lib):
    """Unknown algorithm or staging names are refused before any device call."""
    from paper_2609_40159_amd.api import Plan, UpperPlan
    for cls in (Plan, UpperPlan):
        with pytest.raises(ValueError, match="algo must be one of"):
            cls(None, algo="fast")
        with pytest.raises(ValueError, match="stage_outside must be one of"):
            cls(None, stage_outside="maybe")
