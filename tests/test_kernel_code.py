"""Properties of the compiled stencil code, checked on the host.

The stencil is compiled twice per shape: with ordinary link loads
(`hop_kernel`) and with non-temporal ones (`hop_kernel_nt`, for link fields
that cannot stay in the Infinity Cache).  For FP16 the hinted kernels must be
the ordinary ones with only the hint bits added: then both give the same
bits, and what the parity tests establish for one holds for the other.  (A
version that loaded the hinted FP16 links as float vectors broke this: the
compiled code reused the registers of some link words while their loads were
still in flight.)  The check compiles the stencil source to gfx950 assembly
with the library's own flags and compares the two kernels of every FP16
shape instruction by instruction, branch label numbers aside.

The CG vector update likewise has a variant that reads and writes the inner
solution with the hint, chosen per launch from the size of all its items'
vectors; that is sound only while the two variants do the same floating-point
arithmetic, which the second check compares.

The third check reads every stencil and vector kernel, Wilson and staggered,
for the failure itself:
a register written while a global load that fills it is still outstanding.
"""

import os
import re
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2409_03030_amd import build as B


def _hipcc():
    try:
        return B._hipcc()
    except RuntimeError:
        return None


def _asm(hipcc, folder, src):
    out = os.path.join(folder, src + ".s")
    flags = [f for f in B.HIPFLAGS if not f.startswith("-W")]
    cmd = [hipcc, *flags, "--cuda-device-only", "-x", "hip", "-S", os.path.join(B.CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    with open(out) as f:
        return f.read().split("\n")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    """gfx950 assembly of the sources with non-temporal loads, compiled in parallel."""
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    folder = str(tmp_path_factory.mktemp("asm"))
    srcs = ("hop.hip", "blas.hip", "stag.hip")
    with ThreadPoolExecutor(len(srcs)) as ex:
        return dict(zip(srcs, ex.map(lambda s: _asm(hipcc, folder, s), srcs)))


@pytest.fixture(scope="module")
def hop_asm(asm):
    return asm["hop.hip"]


@pytest.fixture(scope="module")
def blas_asm(asm):
    return asm["blas.hip"]


@pytest.fixture(scope="module")
def stag_asm(asm):
    return asm["stag.hip"]


def _kernels(lines):
    """Instruction lists of every function, branch label numbers removed."""
    funcs, cur, buf = {}, None, []
    for line in lines:
        m = re.match(r"^(_Z\S+):\s*(;.*)?$", line)
        if m:
            cur, buf = m.group(1), []
            continue
        if cur and line.startswith(".Lfunc_end"):
            funcs[cur] = buf
            cur = None
            continue
        s = line.strip()
        if cur and s and not s.startswith(";") and not s.startswith("."):
            buf.append(re.sub(r"\.LBB\d+_", ".LBB_", s))
    return funcs


def _name(nt, prec, recon, mode, split):
    base = "13hop_kernel_nt" if nt else "10hop_kernel"
    return f"_ZN2wd{base}ILi{prec}ELi{recon}ELi{mode}ELi{split}EEEvNS_6LaunchE"


def test_fp16_hinted_kernels_equal_ordinary_ones(hop_asm):
    funcs = _kernels(hop_asm)
    checked = 0
    for recon in (12, 18):
        for mode in (0, 1, 2):
            for split in (1, 2, 4, 8):
                plain = funcs[_name(False, 2, recon, mode, split)]
                hinted = funcs[_name(True, 2, recon, mode, split)]
                nt_loads = sum(1 for s in hinted if s.startswith("global_load") and s.endswith(" nt"))
                assert nt_loads >= 8, (recon, mode, split, nt_loads)
                stripped = [s[:-3] if s.endswith(" nt") else s for s in hinted]
                assert stripped == plain, (recon, mode, split)
                checked += 1
    assert checked == 24


_FP_OPS = re.compile(r"^v_(pk_)?(fma|fmac|mul|add|sub|subrev|cvt|div|rcp|sqrt|max|min)\S*_f(16|32|64)")


def test_cg_update_hint_keeps_its_arithmetic(blas_asm):
    """blas_kernel<P, BLAS_CGUPD, XNT>: the same floating-point instructions
    (as a multiset) with and without the hint on x, at each precision."""
    funcs = _kernels(blas_asm)
    for prec in (0, 1, 2):
        ops = []
        for xnt in (0, 1):
            body = funcs[f"_ZN2wd11blas_kernelILi{prec}ELi1ELb{xnt}EEEvNS_6LaunchE"]
            ops.append(sorted(s.split()[0] for s in body if _FP_OPS.match(s)))
        assert len(ops[0]) > 20, prec
        assert ops[0] == ops[1], prec


def _outstanding_overwrites(body):
    """Instructions that write a register while a global load into it is
    still outstanding: no s_waitcnt vmcnt since the load has retired it
    (vector loads and stores retire in issue order and both count in vmcnt).
    A straight-line reading of the listing: across branches it can only err
    towards reporting more."""
    pend, bad = [], []
    for s in body:
        if s.startswith("s_waitcnt"):
            m = re.search(r"vmcnt\((\d+)\)", s)
            if m:
                k = int(m.group(1))
                pend = pend[len(pend) - k:] if 0 < k < len(pend) else ([] if k == 0 else pend)
            continue
        parts = s.replace(",", " ").split()
        op = parts[0]
        if op.startswith("s_") or len(parts) < 2:
            continue
        is_store = op.startswith(("global_store", "buffer_store", "global_atomic"))
        dst = set()
        if not is_store:
            m = re.match(r"v\[(\d+):(\d+)\]$", parts[1])
            if m:
                dst = set(range(int(m.group(1)), int(m.group(2)) + 1))
            else:
                m = re.match(r"v(\d+)$", parts[1])
                dst = {int(m.group(1))} if m else set()
        if any(dst & r for r, _ in pend):
            bad.append(s)
        if op.startswith(("global_load", "buffer_load")):
            pend.append((dst, s))
        elif is_store:
            pend.append((set(), s))
    return bad


def test_no_register_rewritten_under_an_outstanding_load(hop_asm, blas_asm, stag_asm):
    """Every Wilson and staggered stencil and CG vector kernel (all the
    kernels with non-temporal loads): no instruction writes a register that
    an outstanding global load is still to fill (the failure of the
    float-vector FP16 link loads)."""
    checked = 0
    for asm in (hop_asm, blas_asm, stag_asm):
        for name, body in _kernels(asm).items():
            if not any(k in name for k in ("hop_kernel", "blas_kernel", "stag_kernel", "sblas_kernel")):
                continue
            assert _outstanding_overwrites(body) == [], name
            checked += 1
    assert checked >= 144 + 108
