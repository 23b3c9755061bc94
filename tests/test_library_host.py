"""Host-side checks of the C-ABI library (no GPU work): it loads, exports
every entry point declared in include/vie.h, and its memory model matches
the unknowns memory printed in the paper (Tables III, V, VII, VIII)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    try:
        import paper_1902_02196_amd as vie
    except ImportError as e:
        pytest.skip(str(e))
    return vie


def test_exports_every_declared_symbol():
    vie = _lib()
    hdr = open(os.path.join(ROOT, "include", "vie.h")).read()
    declared = set(re.findall(r"\b(vie_[a-z_0-9]+)\s*\(", hdr))
    import ctypes
    lib = ctypes.CDLL(vie.LIB_PATH)
    missing = [s for s in declared if not hasattr(lib, s)]
    assert not missing, missing
    assert declared == set(vie.EXPORTED)


def _rows():
    rows = []
    for line in open(os.path.join(ROOT, "tests", "golden", "unknowns_memory.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            nx, ny, nz, dofs, mem = line.split()
            rows.append((int(nx), int(ny), int(nz), float(dofs), float(mem)))
    return rows


def test_unknowns_memory_matches_paper_tables():
    vie = _lib()
    for nx, ny, nz, dofs, mem in _rows():
        b = vie.unknowns_bytes_paper(nx, ny, nz)
        assert round(b / 2 ** 30, 3) == pytest.approx(mem, abs=1e-9), (nx, ny, nz)
        # DoFs: 12 unknowns per voxel (Sec. III-A), printed to the table's digits
        digits = len(str(dofs).split(".")[1]) if "." in str(dofs) else 0
        assert round(12 * nx * ny * nz / 1e6, digits) == pytest.approx(dofs, abs=1e-9)


def test_pwc_unknowns_memory_matches_paper_tables():
    """The PWC rows of Tables III, V, VII and VIII: 3 unknowns per voxel
    (Sec. V), 24 N_V complex128 numbers."""
    vie = _lib()
    rows = []
    for line in open(os.path.join(ROOT, "tests", "golden", "unknowns_memory_pwc.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            nx, ny, nz, dofs, mem = line.split()
            rows.append((int(nx), int(ny), int(nz), dofs, float(mem)))
    assert len(rows) == 16
    for nx, ny, nz, dofs, mem in rows:
        b = vie.unknowns_bytes_basis(nx, ny, nz, 3)
        assert round(b / 2 ** 30, 3) == pytest.approx(mem, abs=1e-9), (nx, ny, nz)
        digits = len(dofs.split(".")[1]) if "." in dofs else 0
        assert round(3 * nx * ny * nz / 1e6, digits) == pytest.approx(float(dofs), abs=1e-9), (nx, ny, nz)
        assert vie.unknowns_bytes_basis(nx, ny, nz, 12) == 4 * b == vie.unknowns_bytes_paper(nx, ny, nz)
    assert vie.unknowns_bytes_basis(4, 4, 4, 5) == 0


def test_footprint_model_counts_basis_and_buffers():
    vie = _lib()
    n = 64
    V = n ** 3
    f64 = vie.footprint_bytes(n, n, n, 1, vie.SOLVE_FP64, 50)
    f32 = vie.footprint_bytes(n, n, n, 1, vie.SOLVE_FP32_IR, 50)
    # the Krylov basis dominates: 51 vectors of 12 V complex numbers
    assert f64 > 51 * 12 * V * 16
    assert f32 > 51 * 12 * V * 8
    assert f32 < f64
    f64_4 = vie.footprint_bytes(n, n, n, 4, vie.SOLVE_FP64, 50)
    assert f64_4 > 3 * 51 * 12 * V * 16
    with pytest.raises(vie.VieError):
        vie.footprint_bytes(0, n, n, 1, vie.SOLVE_FP64, 50)
