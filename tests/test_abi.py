"""The C ABI without a GPU: every function include/gw.h declares is exported
by libgwmi.so and bound by the Python layer, and the ctypes structures have
the layout of the C ones (sizes and field offsets, from a host program
compiled against the header)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_2602_06658_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gw.h")


def _declared():
    with open(HEADER) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^\s*(?:gw_status|void|int|const char\s*\*)\s+(gw_\w+)\s*\(", text, re.M)))


def test_header_declares_the_entry_points():
    names = _declared()
    for core in ("gw_create", "gw_set_penalty", "gw_solve", "gw_loss_and_grad", "gw_destroy"):
        assert core in names


def test_library_exports_every_declared_function():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libgwmi.so not built")
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_python_binding_covers_the_header():
    assert set(L.SIGNATURES) == set(_declared())


STRUCTS = {
    "gw_params": L.GwParams,
    "gw_result": L.GwResult,
    "gw_request": L.GwRequest,
    "gw_server_stats": L.GwServerStats,
    "gw_profile": L.GwProfile,
    "gw_sgw_result": L.GwSgwResult,
}


def test_struct_layouts_match_the_header():
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as td:
        src, exe = os.path.join(td, "probe.c"), os.path.join(td, "probe")
        with open(src, "w") as fh:
            fh.write("\n".join(lines))
        subprocess.run(["gcc", "-std=c11", "-o", exe, src], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            parts = ln.split()
            got[(parts[0], parts[1])] = int(parts[2])
    for cname, cls in STRUCTS.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_splitmix64_reference_outputs():
    """The seeded-input generator reproduces the published first outputs of
    SplitMix64 from state 0."""
    from workloads import splitmix64_stream

    gen = splitmix64_stream(0)
    assert [next(gen) for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


@pytest.mark.parametrize("n,nl,seed", [(1, 1, 3), (10, 4, 0), (1000, 256, 7000), (5000, 2048, 2 ** 63 + 5),
                                       (300, 512, 11)])
def test_seeded_landmarks_match_the_generator(n, nl, seed):
    """gw_seeded_landmarks (host code, no GPU) gives the subset that the
    SplitMix64 Fisher-Yates generator of the seeded inputs gives."""
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libgwmi.so not built")
    from workloads import splitmix64_landmarks

    got = L.seeded_landmarks(n, nl, seed)
    ref = splitmix64_landmarks(n, nl, seed)
    assert got == ref.tolist()
    assert len(got) == min(n, nl) and len(set(got)) == len(got) and got == sorted(got)
    assert 0 <= got[0] and got[-1] < n


def test_seeded_landmarks_rejects_bad_arguments():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libgwmi.so not built")
    with pytest.raises(L.GWError):
        L.seeded_landmarks(0, 4, 1)
