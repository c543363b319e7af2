"""C ABI checks that need no GPU: the library loads, exports every entry point
declared in include/dlra.h, and rejects invalid problems before touching the
device."""
import ctypes as C
import os
import re

import pytest

from paper_2508_04484_amd import binding as B
from workloads import configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dlra.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|size_t|const char \*)\s*\**\s*([a-z_]+)\s*\(", src,
                       flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_entry_point():
    lib = B.load()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(B.EXPORTS) == names


def test_struct_layouts_match_header():
    # field order and sizes as in include/dlra.h (LP64)
    assert C.sizeof(B.Grid) == 3 * 4 + 4 + 3 * 8
    assert C.sizeof(B.Beam) == 10 * 8
    assert C.sizeof(B.Options) == 9 * 4 + 4 + 9 * 8 + 2 * 4 + 8
    assert C.sizeof(B.Materials) == 3 * 4 + 4 + 5 * 8


def test_workspace_size_scales_with_problem():
    small = B.workspace_size(configs.small_2d())
    big = B.workspace_size(configs.small_2d(nx=64, ny=64))
    assert 0 < small < big


@pytest.mark.parametrize("bad", [
    dict(r=0), dict(r=60, r_max=60), dict(n_steps=0), dict(precision="half"),
    dict(rank_mode="adaptive", r_min=5, r_max=3), dict(collision=5), dict(egrid=9),
])
def test_invalid_options_rejected(bad):
    p = configs.small_2d()
    raw = {k: bad.pop(k) for k in ("collision", "egrid") if k in bad}
    opts = p.options.with_(**bad)
    if opts.precision not in ("fp64", "mixed"):
        o, _ = B.make_options(p.options)
        o.precision = 7
    else:
        o, _ = B.make_options(opts)
    for k, v in raw.items():
        setattr(o, k, v)
    out = C.c_size_t(0)
    rc = B.load().dlra_workspace_size(C.byref(B.make_grid(p.grid)), p.materials.n_mat, 1,
                                      C.byref(o), C.byref(out))
    assert rc == -1
    assert B.load().dlra_last_error()


@pytest.mark.parametrize("n_mat,n_beams,ok", [(12, 1, True), (16, 4, True), (17, 1, False),
                                              (3, 21, True), (3, 22, False), (1, 65, False),
                                              (1, 0, False)])
def test_material_and_beam_limits(n_mat, n_beams, ok):
    # up to 16 base materials (the paper's twelve elements fit), up to 64
    # beams per joint context, at most 64 source columns n_mat * n_beams
    p = configs.small_2d()
    o, _ = B.make_options(p.options)
    out = C.c_size_t(0)
    rc = B.load().dlra_workspace_size(C.byref(B.make_grid(p.grid)), n_mat, n_beams, C.byref(o),
                                      C.byref(out))
    assert (rc == 0) == ok


def test_workspace_size_grows_with_beams():
    p = configs.small_2d()
    assert B.workspace_size(p, 3) > B.workspace_size(p, 1)


def test_init_rejects_null_workspace_without_touching_the_gpu():
    p = configs.small_2d()
    lib = B.load()
    ctx = C.c_void_p(0)
    o, _ = B.make_options(p.options)
    rc = lib.dlra_init(C.byref(B.make_grid(p.grid)), None, 1, None, C.byref(o), None, 0, None,
                       C.byref(ctx))
    assert rc == -1 and not ctx.value


def test_checkpoint_and_flag_calls_reject_null_context():
    lib = B.load()
    n = C.c_size_t(0)
    assert lib.dlra_save(None, None, C.byref(n)) == -1
    assert lib.dlra_load(None, None, 0) == -1
    assert lib.dlra_sync(None) == -1
    assert lib.dlra_set_uncollided(None, 0, 0, None, None) == -1


def test_plan_objective_rejects_bad_arguments_without_touching_the_gpu():
    lib = B.load()
    assert lib.dlra_plan_objective_work(0, 2) == 0
    assert lib.dlra_plan_objective_work(100, 65) == 0
    assert lib.dlra_plan_objective_work(100, 2) >= 100 + 3
    J = C.c_double()
    g = (C.c_double * 2)()
    w = (C.c_double * 2)(1.0, 1.0)
    gp = C.cast(g, C.POINTER(C.c_double))
    wp = C.cast(w, C.POINTER(C.c_double))
    # null device pointers, too small a work space, negative penalty, bad counts
    assert lib.dlra_plan_objective(100, 2, None, wp, None, 1.0, 0.1, None, 10 ** 6, None,
                                   C.byref(J), gp) == -1
    fake = C.c_void_p(16)   # never dereferenced: validation fails first
    assert lib.dlra_plan_objective(100, 2, fake, wp, fake, 1.0, 0.1, fake, 3, None,
                                   C.byref(J), gp) == -1
    assert lib.dlra_plan_objective(100, 2, fake, wp, fake, 1.0, -0.1, fake, 10 ** 6, None,
                                   C.byref(J), gp) == -1
    assert lib.dlra_plan_objective(100, 0, fake, wp, fake, 1.0, 0.1, fake, 10 ** 6, None,
                                   C.byref(J), gp) == -1


def test_a_second_library_path_is_refused(tmp_path):
    # contexts belong to the copy of the library that made them: one copy per
    # process, and asking for another path is an error rather than a silent
    # reuse of the first
    lib = B.load()
    other = tmp_path / "libdlra_other.so"
    other.write_bytes(b"")
    with pytest.raises(RuntimeError):
        B.load(str(other))
    assert B.load() is lib
    assert B.load(B.LIB_PATH) is lib


def test_roof_probe_rejects_bad_arguments_without_touching_the_gpu():
    lib = B.load()
    out = C.c_double(0.0)
    assert lib.dlra_roof_probe(4, 10, C.byref(out)) == -1
    assert lib.dlra_roof_probe(-1, 10, C.byref(out)) == -1
    assert lib.dlra_roof_probe(0, 0, C.byref(out)) == -1
    assert lib.dlra_roof_probe(0, 10, None) == -1
