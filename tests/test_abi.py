"""The C ABI without a GPU: the library loads, exports every entry point the
header declares, and rejects bad scenes on the host."""
import ctypes
import re
import os

import numpy as np
import pytest

from paper_2603_15186_amd import hgs
from paper_2603_15186_amd.synth import make_random_box, make_floorplan, build_hierarchy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "hgs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hgs_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = hgs.load_library()
    names = declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(n for n, _, _ in hgs.EXPORTS) == names


def test_binding_constants_match_header():
    src = open(os.path.join(ROOT, "include", "hgs.h")).read()
    found = re.findall(r"#define (HGS_[A-Z0-9_]+) +\(?(-?\d+)\)?", src)
    assert len(found) >= 20
    for name, val in found:
        assert getattr(hgs, name) == int(val), name


def test_stats_struct_matches_header_fields():
    src = open(os.path.join(ROOT, "include", "hgs.h")).read()
    body = src[src.index("typedef struct {\n    int64_t cut_size;"):src.index("} hgs_stats;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in re.findall(r"(?:int64_t|double) ([^;]+);", body):
        names += [n.strip() for n in decl.split(",")]
    assert [n for n, _ in hgs.hgs_stats._fields_] == names


def test_plan_struct_matches_header_fields():
    src = open(os.path.join(ROOT, "include", "hgs.h")).read()
    body = src[src.index("typedef struct {\n    int32_t batch_depth;"):src.index("} hgs_plan;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = [n.strip() for d in re.findall(r"(?:int32_t|double) ([^;]+);", body) for n in d.split(",")]
    assert [n for n, _ in hgs.hgs_plan._fields_] == names
    assert ctypes.sizeof(hgs.hgs_plan) == 4 * 4 + 2 * 8 + 6 * 4


def test_slice_grid_struct_matches_header():
    assert ctypes.sizeof(hgs.hgs_slice_grid) == 3 * 8 + 4 * 4 + 8
    assert [n for n, _ in hgs.hgs_slice_grid._fields_] == ["x0", "y0", "cell", "nx", "ny", "n_planes", "rho_min",
                                                           "heights"]


def test_binding_struct_sizes_match_header_layout():
    import ctypes
    assert ctypes.sizeof(hgs.hgs_gaussians) == 8 + 4 + 4 + 5 * 8
    assert ctypes.sizeof(hgs.hgs_hierarchy) == 8 + 4 * 8 + 4 + 4 + 8
    assert ctypes.sizeof(hgs.hgs_camera) == 4 * 2 + 4 * 4 + 12 + 36 + 4 + 12
    assert ctypes.sizeof(hgs.hgs_output) == 24


def test_validation_accepts_good_scenes():
    assert hgs.validate_scene(make_random_box(500, seed=1)) == (0, "")
    leaves, _ = make_floorplan(3000, (6.0, 5.0), 1, 3.0, 8, 2, seed=3)
    assert hgs.validate_scene(build_hierarchy(leaves))[0] == 0


@pytest.mark.parametrize("field,index,value,code", [
    ("scales", (3, 1), 0.0, hgs.HGS_E_INVALID),
    ("scales", (3, 1), np.nan, hgs.HGS_E_INVALID),
    ("means", (7, 2), np.inf, hgs.HGS_E_INVALID),
    ("opacity", (2,), 0.0, hgs.HGS_E_INVALID),
    ("opacity", (2,), 1.5, hgs.HGS_E_INVALID),
    ("quats", (4,), 0.0, hgs.HGS_E_INVALID),
])
def test_validation_rejects_bad_gaussians(field, index, value, code):
    s = make_random_box(50, seed=2)
    getattr(s, field)[index] = value
    st, msg = hgs.validate_scene(s)
    assert st == code and msg


@pytest.fixture()
def hier():
    leaves, _ = make_floorplan(2000, (6.0, 5.0), 1, 3.0, 6, 1, seed=4)
    return build_hierarchy(leaves)


def test_validation_rejects_broken_hierarchies(hier):
    h = hier
    k = int(h.level_offset[2]) + 3
    cases = []
    a = h.parent.copy(); a[k] = int(h.level_offset[2]) + 1; cases.append(("parent", a))
    a = h.child_count.copy(); a[1] = -1; cases.append(("child_count", a))
    a = h.first_child.copy(); a[1] += 1; cases.append(("first_child", a))
    a = h.level_offset.copy(); a[-1] -= 1; cases.append(("level_offset", a))
    a = h.parent.copy(); a[0] = 5; cases.append(("parent", a))
    for field, arr in cases:
        old = getattr(h, field)
        setattr(h, field, arr)
        st, msg = hgs.validate_scene(h)
        setattr(h, field, old)
        assert st == hgs.HGS_E_BAD_HIERARCHY, (field, st, msg)
    b = h.bound.copy(); b[9, 3] = -1.0
    old = h.bound; h.bound = b
    st, _ = hgs.validate_scene(h)
    h.bound = old
    assert st == hgs.HGS_E_INVALID


def test_backward_structs_match_header():
    src = open(os.path.join(ROOT, "include", "hgs.h")).read()
    for name, fields in (("hgs_image_grad", ["rgb", "depth", "alpha"]),
                         ("hgs_scene_grad", ["means", "scales", "quats", "opacity", "sh"])):
        end = src.index("} " + name + ";")
        body = src[src.rindex("typedef struct {", 0, end):end]
        assert re.findall(r"\*\s*([a-z_]+);", body) == fields, name
        st = getattr(hgs, name)
        assert [n for n, _ in st._fields_] == fields
        assert ctypes.sizeof(st) == 8 * len(fields)
