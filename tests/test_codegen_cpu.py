"""Checks on the compiled gfx950 code that no CPU run of the kernels can show.

A chunk loop that prefetches the next chunk into registers only hides the
load latency if those loads are still in flight when the current chunk's
MFMAs issue.  The compiler waits for a load (`s_waitcnt vmcnt(N)`: all but the
N most recent vector-memory operations done) before the first instruction that
reads its result or overwrites its register.  These tests compile the GEMM
sources to device assembly with the library's own flags and, for every global
load that reaches an MFMA with no barrier in between, check whether the load
is waited for before that MFMA.  They also count the exec-mask saves and
branches between consecutive MFMAs: a product behind a branch costs a wait for
every outstanding LDS read.  Every kernel of every source is also checked for
register spills, scratch memory and its static LDS size."""
import os
import re
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_1708_03340_amd import build as B

pytestmark = pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not found")

_VMEM = re.compile(r"^\s*(global_|buffer_|flat_)(load|store|atomic)")
_WAIT = re.compile(r"vmcnt\((\d+)\)")


def _asm(tmp, src):
    out = os.path.join(tmp, src + ".s")
    flags = [f for f in B.COMMON if f != "-fPIC"]
    r = subprocess.run([B.HIPCC, *flags, "--cuda-device-only", "-S", os.path.join(B.CSRC, src), "-o", out],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    with open(out) as f:
        return f.read().split("\n")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    tmp = str(tmp_path_factory.mktemp("asm"))
    srcs = [f for f in B.SOURCES if f.endswith(".hip")]
    with ThreadPoolExecutor(len(srcs)) as ex:
        return dict(zip(srcs, ex.map(lambda s: _asm(tmp, s), srcs)))


def _kernels(lines, kernel):
    """{mangled name: body lines} for every instance of `kernel`."""
    out = {}
    head = re.compile(r"^(_Z\w*" + kernel + r"I\w*):")
    for i, l in enumerate(lines):
        m = head.match(l)
        if m and m.group(1) not in out:
            j = i + 1
            while j < len(lines) and not lines[j].startswith(".Lfunc_end"):
                j += 1
            out[m.group(1)] = lines[i:j]
    return out


def prefetch_waits(body):
    """(loads that reach an MFMA with no barrier between, those among them
    waited for before that MFMA)."""
    total = waited = 0
    for j, x in enumerate(body):
        if not re.match(r"^\s*global_load", x):
            continue
        after, k, w = 0, j + 1, False
        while k < len(body) and "v_mfma" not in body[k] and "s_barrier" not in body[k]:
            if _VMEM.match(body[k]):
                after += 1
            m = _WAIT.search(body[k])
            if m and after >= int(m.group(1)):
                w = True
            k += 1
        if k < len(body) and "v_mfma" in body[k]:
            total += 1
            waited += w
    return total, waited


def test_checker_sees_a_wait():
    # a load whose value the next instruction needs, then an MFMA
    body = ["\tglobal_load_dwordx2 v[0:1], v[2:3], off", "\ts_waitcnt vmcnt(0)",
            "\tv_mfma_f64_16x16x4_f64 v[4:11], v[0:1], v[0:1], v[4:11]"]
    assert prefetch_waits(body) == (1, 1)
    # two loads, only the older one waited for
    body = ["\tglobal_load_dwordx2 v[0:1], v[2:3], off", "\tglobal_load_dwordx2 v[12:13], v[2:3], off",
            "\ts_waitcnt vmcnt(1)", "\tv_mfma_f64_16x16x4_f64 v[4:11], v[0:1], v[0:1], v[4:11]"]
    assert prefetch_waits(body) == (2, 1)
    # a barrier in between: not a prefetch of the MFMA's chunk loop
    body = ["\tglobal_load_dwordx2 v[0:1], v[2:3], off", "\ts_barrier",
            "\tv_mfma_f64_16x16x4_f64 v[4:11], v[0:1], v[0:1], v[4:11]"]
    assert prefetch_waits(body) == (0, 0)


def test_ring_kernels_keep_prefetch_in_flight(asm):
    ks = _kernels(asm["gemm_sb.hip"], "gemm_sb_ring_kernel")
    assert ks
    for name, body in ks.items():
        total, waited = prefetch_waits(body)
        assert total > 0, name
        assert waited == 0, f"{name}: {waited} of {total} prefetch loads waited for before an MFMA"


def test_split_k_float64_prefetch_in_flight(asm):
    # The loader keeps the next chunk's values raw (operand type, unmasked)
    # until they are stashed after the current chunk's products.  The float64
    # Gram instances (one copy of the chunk loop per wave) still wait for 2 of
    # their 64 prefetch loads; every other float64 instance waits for none.
    ks = _kernels(asm["gemm_rk.hip"], "gemm_rk_kernel")
    f64 = {n: b for n, b in ks.items() if "kernelIddd" in n}
    assert f64
    for name, body in f64.items():
        total, waited = prefetch_waits(body)
        assert total > 0, name
        allowed = 2 if "kernelIdddLi1E" in name else 0
        assert waited <= allowed, f"{name}: {waited} of {total} prefetch loads waited for before an MFMA"


def branches_between_products(body):
    """Exec-mask saves and branches between consecutive MFMAs of one run
    (runs are split where more than 200 lines separate two MFMAs)."""
    idx = [j for j, x in enumerate(body) if "v_mfma" in x]
    n = 0
    for a, b in zip(idx, idx[1:]):
        if b - a <= 200:
            n += sum(("saveexec" in x) or ("s_cbranch" in x) for x in body[a + 1:b])
    return len(idx), n


def _split_k(asm, mode, part):
    ks = _kernels(asm["gemm_rk.hip"], "gemm_rk_kernel")
    # template arguments <A, B, math, mode, KC, KM, PART>
    pat = re.compile(r"kernelIdddLi%dELi\d+ELb[01]ELb%dE" % (mode, int(part)))
    sel = {n: b for n, b in ks.items() if pat.search(n)}
    assert sel
    return sel


def test_son_gramian_products_unbranched(asm):
    for name, body in _split_k(asm, 2, False).items():
        nm, nb = branches_between_products(body)
        assert nm > 0 and nb == 0, f"{name}: {nb} branches between {nm} MFMAs"


def test_gram_products_unbranched(asm):
    # one copy of the Gram loop per wave: each copy's block set is fixed at
    # compile time, so its products run without exec-mask branches
    for name, body in _split_k(asm, 1, False).items():
        nm, nb = branches_between_products(body)
        assert nm > 0 and nb == 0, f"{name}: {nb} branches between {nm} MFMAs"


def test_streamed_and_general_products_unbranched(asm):
    sel = {}
    sel.update(_kernels(asm["gemm_sb.hip"], "gemm_sb_ring_kernel"))
    sel.update(_kernels(asm["gemm_sb.hip"], "gemm_sb_kernel"))
    sel.update({n: b for n, b in _kernels(asm["gemm_rk.hip"], "gemm_rk_kernel").items()
                if re.search(r"kernelI[fd]{3}Li0E", n)})    # general mode: full 128 x 128 result
    assert len(sel) > 20
    for name, body in sel.items():
        nm, nb = branches_between_products(body)
        assert nm > 0 and nb == 0, f"{name}: {nb} branches between {nm} MFMAs"


LDS_BYTES = 160 * 1024   # per workgroup on gfx950


def _metadata(lines):
    """{kernel name: {key: int}} from the code object metadata in the assembly."""
    out = {}
    for blk in "\n".join(lines).split("\n  - ")[1:]:
        m = re.search(r"\.name:\s+(\S+)", blk)
        if not m or ".vgpr_count" not in blk:
            continue
        out[m.group(1)] = {k: int(v) for k, v in re.findall(r"\.(\w+):\s+(\d+)\s*$", blk, re.M)}
    return out


# The split-K Gram instances with float64 rows (four per-wave copies of the
# chunk loop in 256 registers) spill two 64-bit values: 8 registers, at most
# 32 bytes of scratch, one store and one reload of each per chunk in one of
# the four copies.  The Cholesky kernel (its diagonal-block step holds a row,
# the DPP broadcasts of the pivot row and the inverse's column in registers)
# moves 4 registers into accumulation registers, with no scratch memory.
# Every other kernel spills nothing.
SPILL_ALLOWED = re.compile(r"gemm_rk_kernelId[df]dLi1ELi32ELb0ELb0E")
SPILL_TO_ACC = re.compile(r"chol_kernel")


def test_no_spills_scratch_or_lds_overflow(asm):
    n = 0
    for src, lines in asm.items():
        for name, md in _metadata(lines).items():
            n += 1
            if SPILL_ALLOWED.search(name):
                assert md.get("vgpr_spill_count", 0) <= 8, f"{src} {name}: VGPR spills"
                assert md.get("private_segment_fixed_size", 0) <= 32, f"{src} {name}: scratch memory"
                continue
            if SPILL_TO_ACC.search(name):
                assert md.get("vgpr_spill_count", 0) <= 4, f"{src} {name}: VGPR spills"
                assert md.get("private_segment_fixed_size", 0) == 0, f"{src} {name}: scratch memory"
                continue
            assert md.get("vgpr_spill_count", 0) == 0, f"{src} {name}: VGPR spills"
            assert md.get("private_segment_fixed_size", 0) == 0, f"{src} {name}: scratch memory"
            assert md.get("group_segment_fixed_size", 0) <= LDS_BYTES, f"{src} {name}: LDS"
    assert n > 100


def test_metadata_parser_reads_the_fields():
    lines = ["amdhsa.kernels:", "  - .agpr_count:     0", "    .group_segment_fixed_size: 150056",
             "    .name:           k1", "    .private_segment_fixed_size: 16", "    .vgpr_count:     352",
             "    .vgpr_spill_count: 3", "  - .group_segment_fixed_size: 0", "    .name:           k2",
             "    .vgpr_count:     12"]
    md = _metadata(lines)
    assert md["k1"]["group_segment_fixed_size"] == 150056
    assert md["k1"]["vgpr_spill_count"] == 3 and md["k1"]["private_segment_fixed_size"] == 16
    assert md["k2"]["vgpr_count"] == 12 and "vgpr_spill_count" not in md["k2"]


def test_split_k_gram_modes_fit_two_workgroups_per_cu(asm):
    # The split-K launches size their reduction split for two 4-wave
    # workgroups on each CU: 2 waves per SIMD, so at most 256 of the 512
    # unified (arch + accumulation) registers per wave, and half the LDS.
    md = _metadata(asm["gemm_rk.hip"])
    sel = {n: v for n, v in md.items() if re.search(r"kernelI[fd]{3}Li[12]E", n)}
    assert len(sel) >= 32
    for name, v in sel.items():
        assert v["max_flat_workgroup_size"] == 256, name
        assert v["vgpr_count"] <= 256, f"{name}: {v['vgpr_count']} registers"
        assert v["group_segment_fixed_size"] <= LDS_BYTES // 2, name


def test_small_eigensolvers_fit_two_nodes_per_cu(asm):
    # orders <= 64 and <= 96 (the batched workload) run two nodes per CU
    md = _metadata(asm["eig.hip"])
    sel = {n: v for n, v in md.items() if re.search(r"eig_kernelILi(64|96)E", n)}
    assert len(sel) == 2
    for name, v in sel.items():
        waves = v["max_flat_workgroup_size"] // 64
        assert 2 * waves <= 8 and v["vgpr_count"] <= 256, name   # 2 waves per SIMD
        assert 2 * v["group_segment_fixed_size"] <= LDS_BYTES, name
