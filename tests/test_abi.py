"""The C-ABI library loads on the CPU and exports every symbol include/nbody.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nb_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1411_5234_amd import _lib
    return _lib.load()


def test_header_and_binding_agree():
    from paper_1411_5234_amd import _lib
    assert declared_symbols() == sorted(_lib.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_version_and_null_context_errors(lib):
    assert lib.nb_version().decode().count(".") == 2
    assert lib.nb_ctx_destroy(None) == -1
    assert lib.nb_sync(None) == -1
    assert lib.nb_last_error(None) == b"null context"


def test_force_plan_is_pure_and_valid():
    from paper_1411_5234_amd import _lib
    seen = {}
    for prec in ("fp64", "mixed"):
        for nj in (1, 100, 1024, 65536, 1 << 20):
            for m in (1, 7, 64, 1000, 4096, 65536, 1 << 20):
                if m > nj:
                    continue
                p = _lib.force_plan(nj, m, prec)
                assert p == _lib.force_plan(nj, m, prec)
                il, s, b = p
                assert il in (1, 2, 4) and s in (1, 4, 16, 64) and 1 <= b <= 1024
                # every lane still walks a useful number of j-bodies
                assert nj // (s * b) >= min(128, nj // (s * b) if s * b > 1 else nj)
                seen[(prec, nj, m)] = p
    # the whole system active at N = 2^20: broadcast LDS reads (S = 1), two
    # i-bodies per lane, and only a small j-split
    il, s, b = seen[("mixed", 1 << 20, 1 << 20)]
    assert (il, s) == (2, 1) and b <= 4
    # a small block in a large system is split across j (the paper's Bfactor)
    il, s, b = seen[("mixed", 65536, 64)]
    assert s * b > 1


def test_force_plan_lane_target():
    """The plan's lane target: 0 and the default give nb_force_plan's plan; a smaller
    target never takes more lanes (i-groups x lanes per i-body x j-chunks); targets
    outside the documented range are refused."""
    from paper_1411_5234_amd import _lib
    default = 1 << 21
    for prec in ("fp64", "mixed"):
        for nj in (1, 300, 4096, 32768, 1 << 20):
            for m in (1, 5, 20, 100, 1000, 4096, 1 << 20):
                if m > nj:
                    continue
                base = _lib.force_plan(nj, m, prec)
                assert _lib.force_plan(nj, m, prec, 0) == base
                assert _lib.force_plan(nj, m, prec, default) == base
                prev = None
                for lanes in (1 << 24, default, 1 << 18, 1 << 14, 1 << 10):
                    il, s, b = _lib.force_plan(nj, m, prec, lanes)
                    assert il in (1, 2, 4) and s in (1, 4, 16, 64) and 1 <= b <= 1024
                    used = -(-m // il) * s * b
                    if prev is not None:
                        assert used <= prev
                    prev = used
    # a small block of a mid-sized system: the default splits it far more than a
    # target sized for a batch of systems does
    il, s, b = _lib.force_plan(32768, 100, "mixed")
    il2, s2, b2 = _lib.force_plan(32768, 100, "mixed", 1 << 14)
    assert s * b > s2 * b2
    for bad in (-1, 1, (1 << 10) - 1, (1 << 24) + 1):
        with pytest.raises(_lib.NbError):
            _lib.force_plan(1024, 10, "mixed", bad)


def test_struct_layouts_match_the_header(tmp_path):
    """ctypes mirrors of nb_system / nb_batch_item / nb_hermite6 / nb_tidal_item /
    nb_nearest_item have the C sizes and offsets."""
    import ctypes
    import subprocess
    from paper_1411_5234_amd import _lib
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "nbody.h"\n'
        'int main(void) { printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", '
        'sizeof(nb_system), '
        'sizeof(nb_batch_item), offsetof(nb_batch_item, status), offsetof(nb_batch_item, eps), '
        'offsetof(nb_batch_item, m), offsetof(nb_batch_item, done), sizeof(nb_hermite6), '
        'offsetof(nb_hermite6, axp32), sizeof(nb_tidal_item), offsetof(nb_tidal_item, m), '
        'offsetof(nb_tidal_item, eps), offsetof(nb_tidal_item, status), '
        'sizeof(nb_nearest_item), offsetof(nb_nearest_item, row_end), '
        'offsetof(nb_nearest_item, dt_cap), offsetof(nb_nearest_item, status)); return 0; }\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    B = _lib.NbBatchItem
    H = _lib.NbHermite6
    Ti = _lib.NbTidalItem
    want = [ctypes.sizeof(_lib.NbSystem), ctypes.sizeof(B), B.status.offset, B.eps.offset,
            B.m.offset, B.done.offset, ctypes.sizeof(H), H.axp32.offset, ctypes.sizeof(Ti),
            Ti.m.offset, Ti.eps.offset, Ti.status.offset, ctypes.sizeof(_lib.NbNearestItem),
            _lib.NbNearestItem.row_end.offset, _lib.NbNearestItem.dt_cap.offset,
            _lib.NbNearestItem.status.offset]
    assert got == want
