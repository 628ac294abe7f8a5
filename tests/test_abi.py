"""The C ABI without a GPU: the library builds for gfx950, exports every function the header
declares, and rejects invalid arguments before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2508_15522_amd import build, gridff
    if not os.path.exists(gridff.LIB_PATH):
        build.build()
    return gridff.lib()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gridff.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gff_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 30
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    from paper_2508_15522_amd import gridff
    assert set(gridff.EXPORTS) <= set(names)


def test_status_strings(lib):
    lib.gff_status_string.restype = C.c_char_p
    assert lib.gff_status_string(0) == b"ok"
    assert lib.gff_status_string(-1) == b"invalid argument"
    assert lib.gff_status_string(-4) == b"workspace too small"


def test_invalid_arguments_rejected_without_device(lib):
    from paper_2508_15522_amd import gridff as G
    assert lib.gff_relax_batch(None, None, None, None, None, None, None, None, None, None) == -1
    assert lib.gff_eval_forces(None, None, None, 0, None, None, None, None, None, None) == -1
    assert lib.gff_plan_create(None, 1, None, None, None) == -1
    assert lib.gff_propose_uniform(C.c_int(4), C.c_int(17), C.c_uint64(1), C.c_uint32(0), C.c_float(3.0),
                                   C.c_float(5.0), None, None, None) == -1
    assert lib.gff_decode_dof(C.c_int(-1), None, C.c_int(0), C.c_float(0), C.c_float(1), None, None) == -1
    assert lib.gff_mlp_create(0, None, None) == -1
    assert lib.gff_refill(None, None, None, C.c_float(0.05), C.c_float(0.1), None, None) == -1
    assert lib.gff_relax_occupancy(None, None, 2, None, None) == -1
    assert lib.gff_dedupe_rmsd_noalloc(None, None, None, C.c_float(0.1), C.c_float(1.0), C.c_float(1.0), 0, 24,
                                       None, None, None, None, None, None) == -1
    g = G.Grid(5, 8, 8, 8, 0, 0, 0, 0.1, 0.1, 0.1, None, None)      # unknown storage
    assert lib.gff_interp_points(C.byref(g), 1, None, None, None, None, None) == -1
    spec = G.grid_spec(3, 8, 8, 0.0, 0.0, 1.0, 0.1)                # nx < 4
    lib.gff_grid_bytes.restype = C.c_size_t
    assert lib.gff_grid_bytes(C.byref(spec), 0) == 0
    spec = G.grid_spec(8, 8, 8, 0.0, 0.0, 1.0, 0.1)
    # columns of z blocks of 8 nodes starting every 5 padded planes: nz = 8 -> 2 blocks
    assert lib.gff_grid_bytes(C.byref(spec), 0) == 8 * 8 * 16 * 16
    assert lib.gff_grid_bytes(C.byref(spec), 1) == 8 * 8 * 16 * 8
    for nz, blocks in ((4, 1), (5, 1), (6, 2), (11, 3), (150, 30)):
        spec = G.grid_spec(8, 8, nz, 0.0, 0.0, 1.0, 0.1)
        assert lib.gff_grid_bytes(C.byref(spec), 0) == 8 * 8 * 8 * blocks * 16
    # workspace queries are host arithmetic
    lib.gff_fit_workspace_bytes.restype = C.c_size_t
    assert lib.gff_fit_workspace_bytes(C.byref(spec)) > 0
    lib.gff_mlp_n_params.restype = C.c_size_t
    assert lib.gff_mlp_n_params(1) == 96 * 256 + 256 + 2 * (256 * 256 + 256) + 41 * 256 + 41 + 32


def test_grid_size_limit_of_buffer_offsets(lib):
    """B-spline grids are read through 32-bit buffer offsets: the evaluation calls accept a
    grid of up to 4 GiB - 1 and reject a larger one before any device work (n = 0 here, so
    the stand-in pointers are never dereferenced)."""
    from paper_2508_15522_amd import gridff as G
    fake = C.c_void_p(0x1000)
    scale = C.c_void_p(0x2000)
    # 1024 x 1024 x 86: 144 slots per column, 2.42e9 bytes in F32
    g = G.Grid(G.STORE_F32, 1024, 1024, 86, 0, 0, 0, 0.1, 0.1, 0.1, fake, None)
    assert lib.gff_interp_points(C.byref(g), 0, None, None, None, None, None) == 0
    # 1024 x 1024 x 160: 256 slots per column, exactly 2^32 bytes in F32, half that in F16
    g = G.Grid(G.STORE_F32, 1024, 1024, 160, 0, 0, 0, 0.1, 0.1, 0.1, fake, None)
    assert lib.gff_interp_points(C.byref(g), 0, None, None, None, None, None) == -2
    g = G.Grid(G.STORE_F16, 1024, 1024, 160, 0, 0, 0, 0.1, 0.1, 0.1, fake, scale)
    assert lib.gff_interp_points(C.byref(g), 0, None, None, None, None, None) == 0


def test_soa_layout_helpers_roundtrip():
    from paper_2508_15522_amd import synth as S
    m = S.mol_chain24()
    x = S.place_replicas(m, 3, S.rocksalt_slab(2, 3), 5)
    assert x.shape == (3, 24, 3)
    assert np.all(x[:, :, 2].min(1) >= 3.0 - 1e-6) and np.all(x[:, :, 2].min(1) <= 5.0 + 1e-6)


def test_struct_layouts_match_the_header(tmp_path):
    """Every ctypes mirror of a public struct has the size and field offsets that a C
    compiler gives the declaration in include/gridff.h."""
    import subprocess
    from paper_2508_15522_amd import gridff as G
    pairs = [(G.Substrate, "gff_substrate"), (G.GridSpec, "gff_grid_spec"), (G.Grid, "gff_grid"),
             (G.MolType, "gff_mol_type"), (G.Launch, "gff_launch"), (G.RelaxParams, "gff_relax_params"),
             (G.State, "gff_state")]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gridff.h"', "int main(void) {"]
    for py, c in pairs:
        lines.append(f'    printf("{c} %zu\\n", sizeof({c}));')
        for f in py._fields_:
            lines.append(f'    printf("{c}.{f[0]} %zu\\n", offsetof({c}, {f[0]}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    subprocess.check_call(["gcc", "-std=c11", "-I", inc, str(src), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for py, c in pairs:
        assert int(got[c]) == C.sizeof(py), c
        for f in py._fields_:
            assert int(got[f"{c}.{f[0]}"]) == getattr(py, f[0]).offset, (c, f[0])


def test_scan_target_helpers():
    """Host helpers that lay out scan targets (input preparation, no device)."""
    from paper_2508_15522_amd import scans as SC
    start = [np.array([[0.0, 0.0, 3.0], [1.0, 2.0, 3.5]]), np.array([[5.0, 5.0, 4.0], [6.0, 7.0, 4.2]])]
    held = np.array([1, 0])
    t = SC.detachment_targets(start, held, np.array([1.3, 1.4, 1.5]))
    assert t.shape == (2, 3, 3)
    assert np.allclose(t[0, :, :2], [1.0, 2.0]) and np.allclose(t[1, :, :2], [5.0, 5.0])
    assert np.allclose(t[:, :, 2], [1.3, 1.4, 1.5])
    d = SC.drag_targets(start, held, (1.0, 1.0), 0.1, 4, height=3.3)
    step = 0.1 / np.sqrt(2.0)
    assert np.allclose(d[0, 3], [1.0 + 3 * step, 2.0 + 3 * step, 3.3])
    assert np.allclose(d[1, 0], [5.0, 5.0, 3.3])
    d2 = SC.drag_targets(start, held, (0.0, 2.0), 0.5, 2)
    assert np.allclose(d2[1, 1], [5.0, 5.5, 4.0])
