"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and its closed-form bases (host code) match the oracle's LAPACK
bases.  No GPU is touched."""

import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "kpcg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kp_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import ctypes
    from paper_2501_03377_amd import kpcg
    lib = ctypes.CDLL(kpcg.LIB_PATH)
    declared = _declared()
    assert len(declared) >= 12
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(kpcg.EXPORTS)


def test_version_and_strerror():
    from paper_2501_03377_amd import kpcg
    assert "kpcg" in kpcg.kp_version()
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert kpcg.kp_strerror(code) != "unknown status"


@pytest.mark.parametrize("bc", oracle.BCS)
@pytest.mark.parametrize("n", [3, 4, 5, 8, 17, 64, 96, 129, 256, 512])
def test_closed_form_basis_matches_oracle(n, bc):
    from paper_2501_03377_amd import kp_basis_1d
    Q, lam = kp_basis_1d(n, bc)
    V, lo, _ = oracle.pinv_init((n,), (bc,))
    V, lo = V[0], lo[0]
    assert np.max(np.abs(lam - lo)) < 1e-13 * max(1, n / 64)
    assert np.max(np.abs(Q.T @ Q - np.eye(n))) < 5e-15 * max(1, n / 16)
    L = oracle.laplacian_1d(n, bc)
    assert np.max(np.abs(L @ Q - Q * lam)) < 1e-14 * max(1, n / 16)
    # equal spectral projectors on each eigenvalue cluster
    for value in np.unique(np.round(lo, 9)):
        a = np.abs(lam - value) < 1e-9
        b = np.abs(lo - value) < 1e-9
        assert a.sum() == b.sum()
        assert np.max(np.abs(Q[:, a] @ Q[:, a].T - V[:, b] @ V[:, b].T)) < 1e-12


def test_basis_rejects_bad_input():
    from paper_2501_03377_amd import KpError, kp_basis_1d
    with pytest.raises(KpError):
        kp_basis_1d(2, "D")
    with pytest.raises(KpError):
        kp_basis_1d(5, 7)


def test_smallest_eigenvalue_accuracy():
    # 4 sin^2(theta/2) keeps relative accuracy where 2 - 2 cos(theta) loses it
    from paper_2501_03377_amd import kp_basis_1d
    import math
    _, lam = kp_basis_1d(512, "DN")
    exact = 4 * math.sin(math.pi / (2 * (2 * 512 + 1))) ** 2
    assert abs(lam[0] - exact) / exact < 1e-15


def test_struct_layouts_match_the_header(tmp_path):
    # the ctypes mirrors of the ABI structs have the C compiler's offsets
    import ctypes
    import shutil
    import subprocess
    from paper_2501_03377_amd import kpcg
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    structs = {"kp_result": kpcg.KpResult, "kp_request": kpcg.KpRequest,
               "kp_completion": kpcg.KpCompletion, "kp_server_stats": kpcg.KpServerStats}
    lines = ['#include <cstdio>', '#include <cstddef>',
             f'#include "{os.path.join(ROOT, "include", "kpcg.h")}"', 'int main() {']
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.cpp"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cxx, "-o", str(exe), str(src)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True,
                               text=True).stdout.splitlines():
        cname, field, value = line.split()
        got[(cname, field)] = int(value)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert got[(cname, field)] == getattr(cls, field).offset, (cname, field)


@pytest.mark.parametrize("dims", [(2048, 1024, 1024), (4096, 4096, 128), (2, 8, 8), (8, 8, 2),
                                  (8, 2, 1), (1 << 20, 1 << 11, 1)])
def test_plan_size_limits_are_checked_before_any_device_call(dims):
    # grids of 2^31 or more unknowns (32-bit in-plane indexing), an axis
    # shorter than eq. (3.1) allows (n >= 3; nz = 1 for 2D), or more blocks
    # per right-hand side than the reductions hold, are rejected up front
    from paper_2501_03377_amd.kpcg import KP_EINVAL, kp_plan_create
    rc, _ = kp_plan_create(*dims, (1, 1, 1), 1, 1, None)
    assert rc == KP_EINVAL, dims


@pytest.mark.parametrize("dims", [(20, 32, 32), (32, 32, 40), (528, 16, 16), (16, 18, 1),
                                  (1024, 16, 16)])
@pytest.mark.parametrize("prec", ["i8x7", "i8x6"])
def test_int8_split_plans_need_axes_multiple_of_16_up_to_512(dims, prec):
    # the int8 split products digitise 16 consecutive values per lane and
    # split at most two k-halves of 256 over the waves of a row tile
    from paper_2501_03377_amd.kpcg import KP_EINVAL, PREC, kp_plan_create
    rc, _ = kp_plan_create(*dims, (1, 1, 1), PREC[prec], 1, None)
    assert rc == KP_EINVAL, dims


def test_int8_split_tile_id():
    # every int8 split product runs one kernel; its plans report id 13
    from paper_2501_03377_amd.kpcg import KP_EINVAL, KP_OK, PREC, kp_tile_shape
    for p in ("i8x7", "i8x6"):
        assert kp_tile_shape(13, PREC[p])[0] == KP_OK
        assert kp_tile_shape(0, PREC[p])[0] == KP_EINVAL
    assert kp_tile_shape(13, 6)[0] == KP_EINVAL


def test_async_entry_points_reject_null_arguments():
    # no device work: argument checks only
    import ctypes
    from paper_2501_03377_amd import kpcg
    assert kpcg._lib.kp_poll(None) == kpcg.KP_EINVAL
    assert kpcg._lib.kp_wait(None) == kpcg.KP_EINVAL
    t = ctypes.c_void_p(123)
    rc = kpcg._lib.kp_solve_async(None, None, None, 1, 1e-10, 10, 0, None, None, ctypes.byref(t))
    assert rc == kpcg.KP_EINVAL and not t.value
    assert kpcg._lib.kp_solve_async(None, None, None, 1, 1e-10, 10, 0, None, None,
                                    None) == kpcg.KP_EINVAL
