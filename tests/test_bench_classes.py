"""bench.py's kernel classes against the kernels compiled into the library
(no GPU): every name a class lists matches a compiled kernel, every
multigrid kernel belongs to the vcycle group and to exactly one of its
classes, and every other kernel of the solve path to exactly one class.
A kernel added to the library without a class would otherwise drop out of
the trace summaries and the counter records unnoticed."""
import re
import shutil
import subprocess

import pytest

import bench
from paper_2411_15897_amd import _native

# kernels no class times: set-up (Galerkin products, coarsest factors,
# Jacobi factors), conversions, copies and fills, the FWI misfit and
# gradient, the single-block solve's cycle start and the power method's
# scaling, the Arnoldi bookkeeping on the small Hessenberg matrices (one
# workgroup per launch, no bandwidth to speak of), and the fine-level X u
# sweep (mode 3) of eh_block_apply
NOT_SOLVE = ("eh::k_cast", "eh::k_copy_strided", "eh::k_dinv", "eh::k_fill", "eh::k_gradient",
             "eh::k_bt_schur", "eh::k_bt_store_inv", "eh::k_bt_couple", "eh::k_gj_", "eh::k_stencil_f64",
             "eh::k_galerkin", "eh::k_dense_from_stencil", "eh::k_sub(", "eh::k_scal(", "eh::k_arn_",
             "eh::k_misfit")
MG_FAMILIES = ("eh::k_fdown<", "eh::k_fup<", "eh::k_gdense<", "eh::k_gstencil<", "eh::k_gfine<",
               "eh::k_gtransfer<", "eh::k_bt_fpart<", "eh::k_bt_chain<", "eh::k_gfine3_lds<",
               "eh::k_gstencil3_lds<", "eh::k_grestrict3_lds<", "eh::k_gprolong3_lds<")


def compiled_kernels():
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm is not available")
    out = subprocess.run([nm, "-C", _native.LIB_PATH], capture_output=True, text=True, check=True).stdout
    names = set()
    for line in out.splitlines():
        m = re.search(r" [VvDdBb] (?:void )?(eh::k_.*)$", line)
        if m:
            names.add("void " + m.group(1))
    assert names, "no kernel symbols found"
    return names


def is_block_apply_sweep(name):
    m = re.match(r"void eh::k_gfine<\w+, \d, \d, (\d)>", name)
    return m is not None and m.group(1) == "3"


def members(cls):
    return bench.CLASS_KERNELS[cls][0]


def test_every_listed_name_is_compiled():
    names = compiled_kernels()
    for cls, (mem, leads) in bench.CLASS_KERNELS.items():
        for pat in tuple(mem) + tuple(leads or ()):
            assert any(pat in n for n in names), (cls, pat)


def test_multigrid_kernels_in_vcycle_and_one_class():
    names = compiled_kernels()
    mg = [n for n in names if any(f in n for f in MG_FAMILIES) and not is_block_apply_sweep(n)]
    assert len(mg) > 100
    for n in mg:
        assert any(p in n for p in members("vcycle")), n
        owners = [c for c in bench.VCYCLE_CLASSES if any(p in n for p in members(c))]
        assert len(owners) == 1, (n, owners)


def test_solve_path_kernels_in_exactly_one_class():
    names = compiled_kernels()
    classes = [c for c in bench.CLASS_KERNELS if c != "vcycle"]
    for n in names:
        if any(x in n for x in NOT_SOLVE) or is_block_apply_sweep(n):
            continue
        owners = [c for c in classes if any(p in n for p in members(c))]
        assert len(owners) == 1, (n, owners)
