"""include/fmm.h is a plain C header: a C11 program that includes it compiles with gcc,
links libfmm.so and gets the documented argument errors (no GPU needed).  The same
program prints the C compiler's layout of every struct in the header and the value of
every constant, and the ctypes binding must agree with both."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2203_07673_amd import _capi as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIP_INCLUDE = "/opt/rocm/include"
needs_toolchain = pytest.mark.skipif(shutil.which("gcc") is None or not os.path.isdir(HIP_INCLUDE),
                                     reason="needs gcc and the HIP headers")

STRUCTS = {"fmm_sparse": C.fmm_sparse, "fmm_batch_graph": C.fmm_batch_graph, "fmm_batch_info": C.fmm_batch_info}
CONSTANTS = ["FMM_ABI_VERSION", "FMM_OK", "FMM_F32", "FMM_BF16", "FMM_F64", "FMM_CSR", "FMM_CSC", "FMM_FUSED",
             "FMM_UNFUSED", "FMM_DC_BF16", "FMM_VARIANT_AUTO", "FMM_VARIANT_DEEP", "FMM_VARIANT_MEDIUM",
             "FMM_VARIANT_SHALLOW", "FMM_BATCH_FWD", "FMM_BATCH_DC_BF16", "FMM_BATCH_BWD", "FMM_GAT_SOFTMAX",
             "FMM_OP_SDDMM", "FMM_OP_SPMM_A", "FMM_OP_SPMM_B",
             "FMM_OP_FUSEDMM_A", "FMM_OP_FUSEDMM_B", "FMM_OP_FUSEDMM_A_BWD", "FMM_OP_FUSEDMM_B_BWD",
             "FMM_OP_SDDMM_BWD", "FMM_OP_SPMM_A_BWD", "FMM_OP_SPMM_B_BWD", "FMM_OP_FUSEDMM_A_BWD_VALUES",
             "FMM_OP_FUSEDMM_B_BWD_VALUES"]


def _program():
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "fmm.h"', "int main(void) {"]
    for name, cls in STRUCTS.items():
        lines.append(f'    printf("size {name} %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'    printf("offset {name}.{field} %zu\\n", offsetof({name}, {field}));')
    for c in CONSTANTS:
        lines.append(f'    printf("const {c} %d\\n", (int){c});')
    lines += [
        "    fmm_sparse d = {0};",
        "    d.orient = FMM_CSC; d.rows = 4; d.cols = 5; d.nnz = 6;",
        '    printf("call abi %d\\n", (int)fmm_abi_version());',
        '    printf("call null %d\\n", (int)fmm_fusedmm_a(NULL, NULL, NULL, 32, FMM_F32, NULL, FMM_FUSED, NULL,'
        ' NULL, 0, NULL));',
        '    printf("call orient %d\\n", (int)fmm_fusedmm_a(&d, (void *)16, (void *)16, 32, FMM_F32, (void *)16,'
        ' FMM_FUSED, NULL, NULL, 0, NULL));',
        '    printf("call status %s\\n", fmm_status_string(FMM_ERR_WORKSPACE));',
        "    return 0;", "}"]
    return "\n".join(lines) + "\n"


@needs_toolchain
def test_header_is_c_and_matches_the_binding(tmp_path):
    lib_dir = os.path.dirname(C.LIB_PATH)
    src = tmp_path / "abi.c"
    src.write_text(_program())
    exe = tmp_path / "abi"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", f"-I{ROOT}/include",
                    f"-I{HIP_INCLUDE}", str(src), "-o", str(exe), f"-L{lib_dir}", "-lfmm",
                    f"-Wl,-rpath,{lib_dir}"], check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=60).stdout.splitlines()
    got = {}
    for line in out:
        kind, key, value = line.split(" ", 2)
        got[(kind, key)] = value
    for name, cls in STRUCTS.items():
        assert int(got[("size", name)]) == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert int(got[("offset", f"{name}.{field}")]) == getattr(cls, field).offset, (name, field)
    for c in CONSTANTS:
        want = C.load().fmm_abi_version() if c == "FMM_ABI_VERSION" else getattr(C, c)
        assert int(got[("const", c)]) == want, c
    assert int(got[("call", "abi")]) == 4
    assert int(got[("call", "null")]) == -1
    assert int(got[("call", "orient")]) == -4   # a CSC descriptor where CSR is required
    assert got[("call", "status")] == C.status_string(-7)


@needs_toolchain
def test_readme_c_example_compiles(tmp_path):
    """The C example in README.md is real code: it compiles as C11 against include/fmm.h
    with every warning an error (compiled only; it would need a GPU to run)."""
    text = open(os.path.join(ROOT, "README.md")).read()
    blocks = text.split("```c\n")
    assert len(blocks) == 2, "README.md holds one C example"
    src = tmp_path / "example.c"
    src.write_text(blocks[1].split("```", 1)[0])
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-Wno-unused-parameter",
                    "-D__HIP_PLATFORM_AMD__", f"-I{ROOT}/include", f"-I{HIP_INCLUDE}", "-c", str(src),
                    "-o", str(tmp_path / "example.o")], check=True, capture_output=True, text=True)
