"""gfx950 code of the force kernels, from this repository's own sources.

The kernel file is compiled to device assembly with the library's flags and
three properties of every force-kernel instantiation are checked:

* the velocity criterion (|R + dtr V|^2, its min with |R|^2) stays behind the
  candidate branch: no basic block holds both the common path's v_rsq_f32
  and the criterion's v_min_f32 (merged, they cost 8 more vector
  instructions on every pair);
* no VGPR or SGPR is spilled and no scratch memory is used;
* the one-i-per-lane kernels, plain and served, fit 6 waves per SIMD (at
  most 80 VGPRs).

No GPU is needed: hipcc cross-compiles for gfx950.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_1205_1222_amd import build

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("isa") / "nb6_kernels.s"
    flags = [f for f in build.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    cmd = [HIPCC, *flags, "--cuda-device-only", "-S", "-o", str(out),
           os.path.join(build.CSRC, "nb6_kernels.hip")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out.read_text()


def _kernels(asm):
    return re.findall(r"^(_ZN3nb6\w*regf\w*):", asm, re.M)


def _body(asm, name):
    start = asm.index("\n" + name + ":")
    return asm[start:asm.index("s_endpgm", start)]


def _meta(asm, name, key):
    # the kernel's entry in the metadata block: its register and scratch
    # fields follow ".name: <symbol>", before the next entry's names
    m = re.search(r"\.name:\s+%s\s(?:(?!\.name:).)*?\.%s:\s+(\d+)" % (re.escape(name), key),
                  asm, re.S)
    assert m is not None, (name, key)
    return int(m.group(1))


def test_every_force_kernel_is_present(asm):
    names = _kernels(asm)
    # 4 coordinate modes x {one-i, two-i, lanes} x {with, without potential}
    # plus the serving kernels: 4 coordinate modes x {one-i, lanes, two-i}
    assert len(names) == 36, names


def test_criterion_stays_behind_its_branch(asm):
    for name in _kernels(asm):
        blocks = re.split(r"\n(?=\.LBB|; %bb\.)", _body(asm, name))
        with_rsq = [b for b in blocks if "v_rsq_f32" in b]
        assert with_rsq, name
        merged = [b for b in with_rsq if "v_min_f32" in b]
        assert not merged, f"{name}: criterion computed on the common path"


def test_no_spills_and_no_scratch(asm):
    for name in _kernels(asm):
        assert _meta(asm, name, "vgpr_spill_count") == 0, name
        assert _meta(asm, name, "sgpr_spill_count") == 0 or "serve" in name, name
        assert _meta(asm, name, "private_segment_fixed_size") == 0, name


def test_one_i_kernel_occupancy(asm):
    for name in _kernels(asm):
        if re.search(r"(?<!serve_)regf_kernelILi\dELi1ELi6E|serve_regf_kernelILi\dELi0E", name):
            assert _meta(asm, name, "vgpr_count") <= 80, name
