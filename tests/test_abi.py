"""The C-ABI library loads on a machine without a GPU, exports every entry
point that include/b3d.h declares, and rejects bad arguments on the host
before touching the device."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "b3d.h")
PROBE_HEADER = os.path.join(ROOT, "include", "b3d_probe.h")


def declared_functions(header=HEADER):
    src = open(header).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(b3d_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_2312_08715_amd as b

    if not os.path.exists(b.LIB_PATH):
        from paper_2312_08715_amd.build import build

        build()
    return b.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("b3d_render_batch", "b3d_score", "b3d_score_backward", "b3d_render_backward", "b3d_c2f_step",
                 "b3d_render_score", "b3d_sample", "b3d_enumerate"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the peak microbenchmarks live in their own library, outside the method's ABI
    from paper_2312_08715_amd import probe

    plib = probe.load_probe_library()
    pnames = declared_functions(PROBE_HEADER)
    assert pnames == ["b3d_probe_fma", "b3d_probe_hbm", "b3d_probe_lds"]
    assert all(hasattr(plib, n) for n in pnames)
    assert not any(hasattr(lib, n) for n in pnames)
    assert plib.b3d_probe_fma(None, 1, 1, None) == -1  # argument errors before any launch


def declared_arity(header=HEADER):
    """Number of parameters of each function the header declares."""
    src = re.sub(r"/\*.*?\*/", "", open(header).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"^\s*(?:const\s+)?\w+\**\s+\**(b3d_\w+)\s*\(([^)]*)\)\s*;", src, flags=re.M):
        params = m.group(2).strip()
        out[m.group(1)] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_binding_signatures_match_the_header(lib):
    # every function the Python binding declares takes as many arguments as
    # the C declaration (a mismatch would only show as a ctypes error on a GPU)
    import paper_2312_08715_amd as b

    arity = declared_arity()
    assert set(b._SIGNATURES) <= set(arity), sorted(set(b._SIGNATURES) - set(arity))
    bad = {n: (len(args), arity[n]) for n, (args, _) in b._SIGNATURES.items() if len(args) != arity[n]}
    assert not bad, bad


def test_host_side_validation_without_a_device(lib):
    import paper_2312_08715_amd as b

    assert b.version().startswith("b3d")
    bad = b.score_params(0.003, 0.0, 1.0, 5)
    rc = lib.b3d_score(None, None, 4, 10, 10, ctypes.byref(bad), None, None, 0, None)
    assert rc == -1 and b"p_out" in lib.b3d_last_error()
    even = b.score_params(0.003, 0.1, 1.0, 4)
    assert lib.b3d_score(None, None, 4, 10, 10, ctypes.byref(even), None, None, 0, None) == -1
    neg = b.score_params(-1.0, 0.1, 1.0, 3)
    assert lib.b3d_score(None, None, 4, 10, 10, ctypes.byref(neg), None, None, 0, None) == -1
    ok = b.score_params(0.003, 0.1, 1.0, 3)
    assert lib.b3d_score(None, None, 0, 10, 10, ctypes.byref(ok), None, None, 0, None) == 0  # N = 0: no-op
    assert lib.b3d_score(None, None, 3, 10, 10, ctypes.byref(ok), None, None, 0, None) == -1  # NULL buffers
    # a workspace smaller than b3d_score_workspace_size is refused before any launch
    nb = ctypes.c_size_t()
    assert lib.b3d_score_workspace_size(10, 12, ctypes.byref(nb)) == 0 and nb.value >= 10 * 12 * 16
    fake = ctypes.c_void_p(16)
    assert lib.b3d_score(fake, fake, 3, 10, 12, ctypes.byref(ok), fake, fake, nb.value - 1, None) == -4
    K = b.intrinsics(100, 100, 50, 40, 80, 100)
    assert lib.b3d_render_batch(None, None, 3, ctypes.byref(K), None, None, None) == -1
    Kbad = b.intrinsics(100, 100, 50, 40, 0, 100)
    assert lib.b3d_unproject(None, 1, ctypes.byref(Kbad), None, None) == -4
    assert lib.b3d_sample(None, 1, 10, 0, 0, 0, 0, None, None, None, None) == -1
    g = b.make_grid(((1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0.5), (0, 0, 0, 1)), (0.01, 0.01, 0.0), (3, 4, 1),
                    n_rot=5)
    assert b.grid_size(g) == 60
    g.count[1] = 0
    assert b.grid_size(g) == 0
    # the tracker's occlusion settings are checked before anything is allocated
    g.count[1] = 4
    stages = (b.Grid * b.B3D_MAX_STAGES)(g)
    fake_meshes = (ctypes.c_void_p * 1)(16)
    P0 = np.eye(4, dtype=np.float32).reshape(16)
    out = ctypes.c_void_p()
    for mv, wd, why in ((1.5, 2.0, b"min_visible"), (-0.1, 2.0, b"min_visible"), (0.2, 0.5, b"widen")):
        tp = b.TrackParams(1, stages, 0, 1e-3, 1e-2, 0.9, 0.999, 1e-8, mv, wd)
        rc = lib.b3d_tracker_create(fake_meshes, 1, ctypes.byref(K), ctypes.byref(ok), ctypes.byref(tp),
                                    P0.ctypes.data, ctypes.byref(out))
        assert rc == -1 and why in lib.b3d_last_error(), (mv, wd, lib.b3d_last_error())
    assert lib.b3d_tracker_state(None, None, None) == -1


def test_mesh_layout_sets_aside_only_faces_no_outside_camera_sees(lib):
    import numpy as np

    import paper_2312_08715_amd as b
    from workloads import box_mesh, make_config, voxel_mesh

    # two touching voxels: their two shared faces (4 triangles) are set aside
    v, t = voxel_mesh(np.array([[0.0, 0.0, 0.0], [0.01, 0.0, 0.0]]))
    info = b.mesh_layout_info(v, t)
    assert info["hidden_pairs"] == 4 and info["drawn"] == 20 and info["dropped"] == 0
    # every face's two halves are paired into a quad: 10 drawn faces, 2 set-aside faces
    assert info["quads"] == 12
    # a two-sided sheet is one component: both sides stay drawn
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], float)
    assert b.mesh_layout_info(v, np.array([[0, 1, 2], [0, 2, 1]]))["hidden_pairs"] == 0
    # a single closed box: nothing set aside; a repeated vertex is dropped
    v, t = box_mesh((0.1, 0.2, 0.3))
    assert b.mesh_layout_info(v, t)["hidden_pairs"] == 0
    t2 = np.vstack([t, [[0, 0, 1]]])
    assert b.mesh_layout_info(v, t2)["dropped"] == 1
    # the voxel blob: every set-aside triangle has a twin with the same corners
    wl = make_config(1)
    info = b.mesh_layout_info(wl.verts, wl.tris)
    assert info["drawn"] + info["hidden_pairs"] + info["dropped"] == wl.tris.shape[0]
    cells = np.round(wl.verts.reshape(-1, 8, 3).mean(1) / 0.01).astype(int)
    occ = {tuple(c) for c in cells}
    shared = sum((tuple(c + d) in occ) for c in cells for d in np.vstack([np.eye(3, dtype=int), -np.eye(3, dtype=int)]))
    assert info["hidden_pairs"] == 2 * shared  # two triangles per touching face, counted from both voxels
    # all voxel faces pair into quads; at most 64 primitives per cluster
    assert info["quads"] * 2 == info["drawn"] + info["hidden_pairs"]
    assert info["clusters"] >= (info["quads"] + 63) // 64
