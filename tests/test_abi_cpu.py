"""Host-side checks of the C ABI: symbols, struct layout, argument validation.

No GPU is needed: every call below fails validation before any HIP work.
"""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1507_00895_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("df.h", "df_mlp.h", "df_lattice.h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(df_\w+)\s*\(", text, re.M))
    return sorted(names)


def test_every_header_is_checked():
    present = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
                     if f.endswith(".h"))
    assert present == sorted(HEADERS)


def test_library_exports_every_declared_symbol():
    lib = B.load()
    decl = declared_functions()
    assert set(decl) == set(B.EXPORTED) | set(B.MLP_EXPORTED) | set(B.LATTICE_EXPORTED)
    for name in decl:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (df_\w+)", out))
    assert set(decl) <= exported


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text('''
#include <stdio.h>
#include <stddef.h>
#include "df.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(df_inst_t), offsetof(df_inst_t, beta),
         offsetof(df_inst_t, g), offsetof(df_inst_t, status), sizeof(df_opts_t),
         offsetof(df_opts_t, max_iter), offsetof(df_opts_t, tol), offsetof(df_opts_t, switch_tol),
         offsetof(df_opts_t, accel), offsetof(df_opts_t, symmetry),
         offsetof(df_opts_t, graph_unroll));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals == [ctypes.sizeof(B.DfInst), B.DfInst.beta.offset, B.DfInst.g.offset,
                    B.DfInst.status.offset, ctypes.sizeof(B.DfOpts), B.DfOpts.max_iter.offset,
                    B.DfOpts.tol.offset, B.DfOpts.switch_tol.offset, B.DfOpts.accel.offset,
                    B.DfOpts.symmetry.offset, B.DfOpts.graph_unroll.offset]


def _inst(**kw):
    base = dict(D=2, nk=8, n_nu=16, n_om=1, beta=10.0)
    base.update(kw)
    fake = 0x1000
    return B.DfInst(base["D"], base["nk"], base["n_nu"], base["n_om"], base["beta"],
                    *([fake] * 11), fake)


@pytest.mark.parametrize("kw,code", [
    (dict(n_om=2), B.DF_E_INVAL),            # even bosonic count
    (dict(n_nu=15), B.DF_E_INVAL),           # odd fermionic count
    (dict(n_om=17), B.DF_E_INVAL),           # n_om > n_nu - 1
    (dict(nk=12), B.DF_E_UNSUPPORTED),       # not a power of two
    (dict(D=5, nk=4), B.DF_E_UNSUPPORTED),
    (dict(D=0), B.DF_E_UNSUPPORTED),
    (dict(D=3, nk=32), B.DF_E_UNSUPPORTED),  # N = 32768 > 4096
    (dict(D=4, nk=16), B.DF_E_UNSUPPORTED),  # N = 65536 > 4096
    (dict(n_nu=130, n_om=3), B.DF_E_UNSUPPORTED),
    (dict(beta=0.0), B.DF_E_INVAL),
])
def test_workspace_size_rejects_bad_shapes(kw, code):
    lib = B.load()
    arr = (B.DfInst * 1)(_inst(**kw))
    n = ctypes.c_size_t(0)
    assert lib.df_workspace_size(arr, 1, None, ctypes.byref(n)) == code


def test_workspace_size_and_validation_order():
    lib = B.load()
    arr = (B.DfInst * 1)(_inst())
    n = ctypes.c_size_t(0)
    assert lib.df_workspace_size(arr, 1, None, ctypes.byref(n)) == B.DF_OK
    assert n.value > 0 and n.value % 256 == 0
    # null / misaligned / short workspace is refused before any device work
    assert lib.df_dual_gf(arr, 1, None, n.value, None) == B.DF_E_WORKSPACE
    assert lib.df_bubble(arr, 1, 0x1001, n.value, None) == B.DF_E_WORKSPACE
    assert lib.df_sigma(arr, 1, 0x1000, n.value - 256, None) == B.DF_E_WORKSPACE
    assert lib.df_dual_gf(arr, 0, 0x1000, n.value, None) == B.DF_E_INVAL
    bad = B.make_opts(mix=0.0)
    assert lib.df_iterate(arr, 1, ctypes.byref(bad), None, None, 0x1000, n.value, None) == B.DF_E_INVAL
    bad = B.make_opts(prec=7)
    assert lib.df_ladder_solve(arr, 1, ctypes.byref(bad), 0x1000, n.value, None) == B.DF_E_INVAL
    # the adaptive schedule belongs to the loop only
    ad = B.make_opts(prec=B.DF_ADAPTIVE)
    assert lib.df_ladder_solve(arr, 1, ctypes.byref(ad), 0x1000, n.value, None) == B.DF_E_INVAL
    assert lib.df_workspace_size(arr, 1, ctypes.byref(ad), ctypes.byref(n)) == B.DF_OK
    bad = B.make_opts(accel=9)
    assert lib.df_ladder_solve(arr, 1, ctypes.byref(bad), 0x1000, n.value, None) == B.DF_E_INVAL
    bad = B.make_opts(symmetry=2)
    assert lib.df_ladder_solve(arr, 1, ctypes.byref(bad), 0x1000, n.value, None) == B.DF_E_INVAL
    assert lib.df_iterate(arr, 1, ctypes.byref(bad), None, None, 0x1000, n.value, None) == B.DF_E_INVAL
    # iterations per captured graph: 0 or 1 (one), up to 64
    for u in (-1, 65):
        bad = B.make_opts(graph_unroll=u)
        assert lib.df_iterate(arr, 1, ctypes.byref(bad), None, None, 0x1000, n.value, None) == B.DF_E_INVAL
    # Anderson history needs workspace
    m0, m5 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.df_workspace_size(arr, 1, ctypes.byref(B.make_opts()), ctypes.byref(m0)) == B.DF_OK
    assert lib.df_workspace_size(arr, 1, ctypes.byref(B.make_opts(accel=5)), ctypes.byref(m5)) == B.DF_OK
    assert m5.value >= m0.value + 13 * 16 * 64 * 16
    assert B.df_strerror(B.DF_E_WORKSPACE).startswith("workspace")
    assert B.df_version() >= 100


def test_workspace_grows_with_instances():
    lib = B.load()
    one = (B.DfInst * 1)(_inst())
    two = (B.DfInst * 2)(_inst(), _inst(D=3, nk=4, n_nu=32, n_om=5))
    a, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.df_workspace_size(one, 1, None, ctypes.byref(a)) == 0
    assert lib.df_workspace_size(two, 2, None, ctypes.byref(b)) == 0
    assert b.value > a.value


def test_mlp_host_validation():
    lib = B._mlp_lib()
    assert B.df_mlp_param_count([5, 7, 3]) == 5 * 7 + 7 + 7 * 3 + 3
    n, dims = B._dims([5, 7, 3])
    size = ctypes.c_size_t(0)
    assert lib.df_mlp_workspace_size(n, dims, 0, ctypes.byref(size)) == B.DF_E_INVAL
    assert lib.df_mlp_workspace_size(n, dims, 10, ctypes.byref(size)) == B.DF_OK
    assert size.value > 0 and size.value % 256 == 0
    bad = (ctypes.c_int32 * 3)(5, 0, 3)
    assert lib.df_mlp_param_count(2, bad, ctypes.byref(size)) == B.DF_E_INVAL
    assert lib.df_mlp_param_count(0, dims, ctypes.byref(size)) == B.DF_E_INVAL
    assert lib.df_mlp_param_count(9, dims, ctypes.byref(size)) == B.DF_E_INVAL
    assert lib.df_mlp_forward(n, dims, None, None, 4, None, None, 0, None) == B.DF_E_INVAL
    fake = 0x1000
    assert lib.df_mlp_forward(n, dims, fake, fake, 4, fake, None, 0, None) == B.DF_E_WORKSPACE
    assert lib.df_mlp_forward(n, dims, fake, fake, 4, fake, fake + 8, 1 << 30, None) == B.DF_E_WORKSPACE
    assert lib.df_mlp_loss_grad(n, dims, fake, fake, None, 4, fake, None, fake, 1 << 30,
                                None) == B.DF_E_INVAL
    assert lib.df_mlp_adam(0, fake, fake, fake, fake, 1, 1e-3, None) == B.DF_E_INVAL
    assert lib.df_mlp_adam(10, fake, fake, fake, fake, 0, 1e-3, None) == B.DF_E_INVAL
    assert lib.df_mlp_adam(10, fake, fake, fake, fake, 1, 0.0, None) == B.DF_E_INVAL


def test_ladder_variant_choice_host_side(tmp_path, monkeypatch):
    B.df_autotune_reset()
    # defaults: the capped builds that measured fastest at n_nu = 64
    assert B.df_ladder_variant(64, B.DF_FP64) == "gjb_o3"
    assert B.df_ladder_variant(64, B.DF_FP32_REFINE) == "mixed_o3"
    assert B.df_ladder_variant(96, B.DF_FP32_REFINE) == "mixed_o3"  # refined kernel up to 128
    assert B.df_ladder_variant(128, B.DF_FP32_REFINE) == "mixed"
    assert B.df_ladder_variant(128, B.DF_FP64) == "gjb"
    assert B.df_ladder_variant(64, B.DF_FP32) == "fp32_o4"
    assert B.df_ladder_variant(128, B.DF_FP32) == "fp32"            # FP32 alone up to 128
    assert B.df_ladder_variant(96, B.DF_FP32) == "fp32"
    with pytest.raises(B.DfError):
        B.df_ladder_variant(64, B.DF_ADAPTIVE)
    B.df_ladder_set_variant(64, B.DF_FP64, "gjb_o4")
    assert B.df_ladder_variant(64, B.DF_FP64) == "gjb_o4"
    assert B.df_ladder_variant(62, B.DF_FP64) == "gjb_o3"            # keyed by exact n_nu
    # persistent grids: the FP64 certified builds with an item loop
    B.df_ladder_set_variant(64, B.DF_FP64, "gjb_o3@p1")
    assert B.df_ladder_variant(64, B.DF_FP64) == "gjb_o3@p1"
    B.df_ladder_set_variant(128, B.DF_FP64, "gjb@p2")
    assert B.df_ladder_variant(128, B.DF_FP64) == "gjb@p2"
    B.df_ladder_set_variant(64, B.DF_FP64, "gjb_o4")
    for bad in [(96, B.DF_FP64, "gjb_o3"), (128, B.DF_FP64, "gjb_o4"), (64, B.DF_FP64, "mixed"),
                (64, B.DF_FP64, "gjb_o4@p1"), (64, B.DF_FP32, "fp32_o4@p1"),
                (64, B.DF_FP64, "vector@p1"), (128, B.DF_FP32_REFINE, "mixed_o3"),
                (128, B.DF_FP32_REFINE, "gjb"), (96, B.DF_FP32_REFINE, "gjb"),
                (64, B.DF_FP32_REFINE, "vector"), (64, B.DF_FP32_REFINE, "fp32_o4"),
                (96, B.DF_FP32_REFINE, "mixed_o4"), (64, B.DF_FP64, "mixed_o3"),
                (64, B.DF_FP32, "mixed"), (64, B.DF_FP64, "fp32_o4"), (96, B.DF_FP32, "fp32_o4"),
                (128, B.DF_FP32, "fp32_o5"), (128, B.DF_FP32, "gjb")]:
        with pytest.raises(B.DfError) as e:
            B.df_ladder_set_variant(*bad)
        assert e.value.code == B.DF_E_UNSUPPORTED
    with pytest.raises(B.DfError):
        B.df_ladder_set_variant(64, B.DF_FP64, "nonsense")
    with pytest.raises(B.DfError):
        B.df_ladder_variant(130, B.DF_FP64)
    B.df_autotune_reset()
    assert B.df_ladder_variant(64, B.DF_FP64) == "gjb_o3"


def test_bubble_noalloc_validates_before_any_gpu_work():
    lib = B.load()
    assert lib.df_bubble_noalloc(None, 1, None) == B.DF_E_INVAL
    arr = (B.DfInst * 1)(_inst())
    assert lib.df_bubble_noalloc(arr, 0, None) == B.DF_E_INVAL
    bad = _inst()
    bad.nk = 6
    assert lib.df_bubble_noalloc((B.DfInst * 1)(bad), 1, None) == B.DF_E_UNSUPPORTED
    nogd = _inst()
    nogd.gd = None
    assert lib.df_bubble_noalloc((B.DfInst * 1)(nogd), 1, None) == B.DF_E_INVAL


def test_autotune_validates_before_any_gpu_work():
    lib = B.load()
    assert lib.df_autotune(None, 1, None, None, 0, None) == B.DF_E_INVAL
    arr = (B.DfInst * 1)(_inst())
    assert lib.df_autotune(arr, 1, None, None, 0, None) == B.DF_E_WORKSPACE


def test_lattice_argument_validation():
    """df_lattice rejects bad instances, mu and workspaces before any HIP work."""
    lib = B._lattice_lib()
    n = ctypes.c_size_t(0)
    good = _inst(n_om=3)
    assert lib.df_lattice_workspace_size(ctypes.byref(good), ctypes.byref(n)) == B.DF_OK
    N, n_nu = 64, 16
    fld = n_nu * N * 16
    chunk = min(2 * N, 512)
    assert n.value >= 7 * fld + 2 * N * 16 + chunk * n_nu * (n_nu + 1) * 16
    assert lib.df_lattice_workspace_size(None, ctypes.byref(n)) == B.DF_E_INVAL
    bad = _inst(n_nu=15)
    assert lib.df_lattice_workspace_size(ctypes.byref(bad), ctypes.byref(n)) == B.DF_E_INVAL
    big = _inst(n_nu=130)
    assert lib.df_lattice_workspace_size(ctypes.byref(big), ctypes.byref(n)) == B.DF_E_UNSUPPORTED
    fake = 0x1000
    args = [fake, fake, fake, fake]
    assert lib.df_lattice(ctypes.byref(good), float("nan"), *args, fake * 256, 1 << 40,
                          None) == B.DF_E_INVAL
    assert lib.df_lattice(ctypes.byref(good), 1.0, *args, None, 1 << 40, None) == B.DF_E_WORKSPACE
    assert lib.df_lattice(ctypes.byref(good), 1.0, *args, fake + 8, 1 << 40,
                          None) == B.DF_E_WORKSPACE
    assert lib.df_lattice(ctypes.byref(good), 1.0, *args, fake * 256, 16, None) == B.DF_E_WORKSPACE
    nog = _inst(n_om=3)
    nog.gamma_uu = None
    assert lib.df_lattice(ctypes.byref(nog), 1.0, *args, fake * 256, 1 << 40,
                          None) == B.DF_E_INVAL
