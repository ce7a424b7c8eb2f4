"""The C ABI from C (CPU only): tests/c/abi_check.c includes include/dop.h as
plain C99, links libdop.so and calls its host-only paths.  Checks that the
header compiles as C, that the dop_problem layout the C compiler sees is the
one the Python binding mirrors field by field, and the workspace sizes and
status codes the C caller gets."""

import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2505_22313_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def c_output(tmp_path_factory):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    so = L.LIB_PATH
    if not os.path.exists(so):
        pytest.skip("libdop.so not built")
    exe = str(tmp_path_factory.mktemp("c") / "abi_check")
    subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c", "abi_check.c"), so,
                    "-Wl,-rpath," + os.path.dirname(so), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    rows = {}
    for line in out.splitlines():
        key, *vals = line.split()
        rows[key] = vals
    return rows


def test_struct_layout_matches_binding(c_output):
    assert int(c_output["sizeof"][0]) == ctypes.sizeof(L.DopProblem)
    for name, _ in L.DopProblem._fields_:
        key = "off_" + ("lambda" if name == "lambda_" else name)
        assert int(c_output[key][0]) == getattr(L.DopProblem, name).offset, name


def test_status_strings(c_output):
    assert c_output["status_ok"] == ["DOP_OK"]
    assert c_output["status_unsupported"] == ["DOP_ERR_UNSUPPORTED"]


def test_workspace_sizes_and_errors(c_output):
    assert c_output["ws_1024"] == ["0", str(8 * 1024 * (1024 + 16))]
    assert c_output["ws_paper"] == ["0", str(8 * 128640 * (85760 + 16))]
    assert int(c_output["ws_1000"][0]) == L.DOP_ERR_UNSUPPORTED
    assert c_output["err_1000_mentions_paper_grid"] == ["1"]
    assert int(c_output["ws_n_gt_m"][0]) == L.DOP_ERR_INVALID_ARG
    assert int(c_output["psf_null_ctx"][0]) == L.DOP_ERR_INVALID_ARG
