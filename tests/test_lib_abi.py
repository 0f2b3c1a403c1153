"""The C interface: the built library loads and exports every function that
the headers declare (no GPU needed, no compute call made)."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = ["include/pi.h", "include/pi_unet.h", "include/pi_flow.h"]
LIBS = {h: "paper_2311_16935_amd/libpi.so" for h in HEADERS}
PREFIX = {"include/pi.h": "pi", "include/pi_unet.h": "pu", "include/pi_flow.h": "pi"}


def declared(header):
    txt = open(os.path.join(ROOT, header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    pre = PREFIX[header]
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(" + pre + r"_\w*)\s*\(", txt, flags=re.M)
    return sorted(set(names))


@pytest.mark.parametrize("header", HEADERS)
def test_library_exports_every_declared_function(header):
    lib_path = os.path.join(ROOT, LIBS[header])
    assert os.path.exists(lib_path), "build the library first (__graft_entry__.build())"
    names = declared(header)
    assert len(names) >= (1 if header.endswith("pi_flow.h") else 8)
    lib = ctypes.CDLL(lib_path)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (p[iu]_\w+)", out))
    assert set(names) <= exported


def test_binding_names_match_header():
    import paper_2311_16935_amd as pi

    names = declared("include/pi.h")
    assert sorted(pi.EXPORTED) == names
    for n in names:
        assert callable(getattr(pi, n))


def test_layer_binding_names_match_header():
    from paper_2311_16935_amd import unet

    names = declared("include/pi_unet.h")
    assert sorted(unet.EXPORTED) == names
    for n in names:
        assert callable(getattr(unet, n))


def test_flow_binding_names_match_header():
    from paper_2311_16935_amd import flow

    names = declared("include/pi_flow.h")
    assert sorted(flow.EXPORTED) == names
    for n in names:
        assert callable(getattr(flow, n))


def test_status_strings_without_gpu():
    import paper_2311_16935_amd as pi

    assert pi.pi_status_string(0) == "ok"
    assert "max_iter" in pi.pi_status_string(4)
    assert pi.pi_status_string(99) == "unknown status"


def test_plan_argument_checks_fail_before_touching_the_device():
    import paper_2311_16935_amd as pi

    for args in [(4, (5, 5), (1.0, 1.0)), (2, (0, 5), (1.0, 1.0)), (2, (5, 5), (1.0, 0.0)),
                 (2, (5, 5), (1.0, float("nan"))), (3, (1 << 11, 1 << 11, 1 << 10), (1.0, 1.0, 1.0))]:
        with pytest.raises(pi.PiError) as e:
            pi.pi_plan(*args)
        assert e.value.status == pi.PI_ERR_INVALID_ARG


def test_cell_centered_flag_checks_fail_before_touching_the_device():
    import paper_2311_16935_amd as pi

    for args in [(3, (5, 5, 5), (1.0, 1.0, 1.0), None, pi.PI_CELL_CENTERED),
                 (2, (5, 5), (1.0, 1.0), None, pi.PI_CELL_CENTERED | pi.PI_INNER_BICGSTAB),
                 (2, (5, 5), (1.0, 1.0), None, 0x10)]:
        with pytest.raises(pi.PiError) as e:
            pi.pi_plan(*args)
        assert e.value.status == pi.PI_ERR_INVALID_ARG


def test_noalloc_size_limit_fails_before_touching_the_device():
    import ctypes

    import paper_2311_16935_amd as pi

    n = pi.PI_NOALLOC_MAX_INSTANCES + 1
    rc = pi.lib.pi_solve_batched_noalloc(n, None, None, None, None, None, None, 10, ctypes.c_uint32(0), None, None)
    assert rc == pi.PI_ERR_TOO_LARGE
    assert "scratch" in pi.pi_status_string(rc)
