"""CPU-side checks of the built library: it loads and exports every symbol
declared in include/pbng.h, and the Python binding mirrors the ABI structs."""
import ctypes
import os
import re
import subprocess
import tempfile

import paper_2110_12511_amd as pb
from paper_2110_12511_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pbng.h")).read()
    return sorted(set(re.findall(r"\b(pbng_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = pb.load()
    names = _declared()
    assert "pbng_count" in names and "pbng_tip" in names and "pbng_wing" in names
    for name in names:
        assert hasattr(lib, name), name


def _c_layout(struct, fields):
    """sizeof and field offsets of a struct of include/pbng.h as the C
    compiler lays it out (gcc on the host)."""
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "pbng.h"', "int main(void) {",
           f'  printf("%zu\\n", sizeof({struct}));']
    src += [f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    src += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        with open(c, "w") as fh:
            fh.write("\n".join(src) + "\n")
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        vals = [int(v) for v in subprocess.check_output([exe]).split()]
    return vals[0], vals[1:]


def test_struct_layouts():
    """The ctypes mirrors of pbng_csr, pbng_opts and pbng_stats have the C
    compiler's size and field offsets."""
    for struct, cls in (("pbng_csr", binding.Csr), ("pbng_opts", binding.Opts), ("pbng_stats", binding.Stats),
                        ("pbng_kernel_stat", binding.KernelStat)):
        fields = [f for f, _ in cls._fields_]
        size, offs = _c_layout(struct, fields)
        assert ctypes.sizeof(cls) == size, struct
        assert [getattr(cls, f).offset for f in fields] == offs, struct


def _c_values(names):
    """Values of header constants (macros and enumerators) as the C compiler
    sees them."""
    src = ["#include <stdio.h>", '#include "pbng.h"', "int main(void) {"]
    src += [f'  printf("%lld\\n", (long long)({n}));' for n in names]
    src += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "consts.c")
        exe = os.path.join(d, "consts")
        with open(c, "w") as fh:
            fh.write("\n".join(src) + "\n")
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        return [int(v) for v in subprocess.check_output([exe]).split()]


def test_constants_match_header():
    """Flags, enumerators, error codes, kernel classes and the parameter
    count of the binding equal include/pbng.h's."""
    pairs = {
        "PBNG_F_NO_DYNAMIC": pb.F_NO_DYNAMIC, "PBNG_F_NO_BATCH": pb.F_NO_BATCH,
        "PBNG_F_NO_DENSE_TILE": pb.F_NO_DENSE_TILE, "PBNG_F_KERNEL_TIMING": binding.F_KERNEL_TIMING,
        "PBNG_F_HOST_ROUNDS": pb.F_HOST_ROUNDS, "PBNG_F_SHORT_PROBE": pb.F_SHORT_PROBE,
        "PBNG_BOUND_PLAIN": pb.BOUND_PLAIN, "PBNG_BOUND_LEARNED": pb.BOUND_LEARNED,
        "PBNG_BOUND_RANDOM": pb.BOUND_RANDOM, "PBNG_BOUND_PAPER": pb.BOUND_PAPER,
        "PBNG_SIDE_U": pb.SIDE_U, "PBNG_SIDE_V": pb.SIDE_V, "PBNG_COUNT_VERTEX_U": pb.COUNT_VERTEX_U,
        "PBNG_COUNT_VERTEX_V": pb.COUNT_VERTEX_V, "PBNG_COUNT_EDGE": pb.COUNT_EDGE,
        "PBNG_K_NCLASS": len(binding.K_NAMES), "PBNG_MLP_NPARAM": binding.MLP_NPARAM,
    }
    names = list(pairs)
    assert _c_values(names) == [pairs[n] for n in names]
    # error codes: the binding's names for them are the header's
    codes = {name: code for code, name in binding.ERRORS.items()}
    assert _c_values(list(codes)) == list(codes.values())
    classes = ["PBNG_K_COUNT", "PBNG_K_TIP_PEEL", "PBNG_K_FD", "PBNG_K_WING_CD", "PBNG_K_DENSE", "PBNG_K_TIP_HRANGE",
               "PBNG_K_TIP_TILED"]
    assert _c_values(classes) == list(range(len(binding.K_NAMES)))


def test_null_context_rejected():
    lib = pb.load()
    assert lib.pbng_count(None, None, 0, None, None) == -1
    assert lib.pbng_tip(None, None, 0, None, None) == -1
    assert lib.pbng_wing(None, None, None, None) == -1
    assert lib.pbng_last_stats(None, None) == -1
