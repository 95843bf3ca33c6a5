"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
function declared in include/aa.h, computes the plan on the host exactly like the
oracle, and rejects bad descriptors with the documented codes."""

import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from synth import dm_plan
from synth.workloads import workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aa.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(aa_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def aa():
    from paper_2101_00941_amd import _native
    return _native


def test_library_exports_every_declared_function(aa):
    L = aa.lib()
    names = _declared()
    assert "aa_plan" in names and "aa_dedisperse" in names and "aa_single_pulse" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert missing == []
    out = subprocess.run(["nm", "-D", "--defined-only", aa.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (aa_\w+)", out))
    assert set(names) <= exported


def _plan(w, **kw):
    from paper_2101_00941_amd import Plan
    return Plan.from_workload(w, host_only=True, **kw)


@pytest.mark.parametrize("name", ["tiny_128ch_32k", "survey_4096ch_1M"])
def test_host_plan_matches_oracle(name):
    w = workload(name)
    p = _plan(w)
    want = oracle.shift_table(w["dms"], w["nchan"], w["f_top"], w["foff"], w["tsamp"])
    assert np.array_equal(p.shifts().astype(np.int64), want)
    sz = oracle.sizes(want, w["nsamp"], w["widths"], w["stat_block"])
    assert p.info["maxshift"] == sz["maxshift"] and p.info["n_dd"] == sz["n_dd"]
    assert p.info["n_start"] == sz["n_start"] and p.info["nblocks"] == sz["nblocks"]
    assert p.info["device"] == -1


def test_host_plan_random_bands():
    rng = np.random.default_rng(0)
    from paper_2101_00941_amd import Plan
    for _ in range(20):
        nchan = int(rng.integers(1, 700))
        foff = float(rng.uniform(0.01, 1.0))
        f_top = float(rng.uniform(nchan * foff + 50, 3000))
        tsamp = float(rng.choice([32e-6, 64e-6, 1e-4, 1.31072e-4]))
        dms = np.sort(rng.uniform(0, 500, int(rng.integers(1, 40))))
        p = Plan(nchan, 1 << 20, f_top, foff, tsamp, dms, [1, 2, 4], 6.0, host_only=True)
        want = oracle.shift_table(dms, nchan, f_top, foff, tsamp)
        assert np.array_equal(p.shifts().astype(np.int64), want)


def test_plan_errors(aa):
    from paper_2101_00941_amd import Plan, AAError
    ok = dict(nchan=64, nsamp=4096, f_top=1500.0, foff=1.0, tsamp=64e-6, dms=[0.0, 1.0], widths=[1, 2],
              threshold=6.0)

    def code(**kw):
        a = dict(ok)
        a.update(kw)
        try:
            Plan(**a, host_only=True)
        except AAError as e:
            return e.code
        return 0

    assert code() == 0
    assert code(dms=[2.0, 1.0]) == aa.AA_EINVAL
    assert code(dms=[-1.0]) == aa.AA_EINVAL
    assert code(foff=-1.0) == aa.AA_EINVAL
    assert code(nchan=2000) == aa.AA_EINVAL               # bottom channel below 0 MHz
    assert code(widths=[2, 1]) == aa.AA_EINVAL
    assert code(widths=[1, 1]) == aa.AA_EINVAL
    assert code(widths=[0]) == aa.AA_EINVAL
    assert code(widths=[2048]) == aa.AA_EINVAL            # wider than AA_MAX_WIDTH
    assert code(stat_block=100) == aa.AA_EINVAL
    assert code(threshold=float("nan")) == aa.AA_EINVAL
    assert code(nsamp=4) == aa.AA_ESHORT
    assert code(dms=[0.0, 5000.0]) == aa.AA_ESHORT       # maxshift beyond nsamp
    assert aa.lib().aa_plan(None, None) == aa.AA_EINVAL
    assert b"null" in aa.lib().aa_last_error()


def test_dedisperse_rejects_host_only_plan(aa):
    p = _plan(workload("tiny_128ch_32k"))
    rc = aa.lib().aa_dedisperse(p.handle, C.c_void_p(256), 32768, 32768, C.c_void_p(256), 32768, None)
    assert rc == aa.AA_EINVAL
    assert b"host-only" in aa.lib().aa_last_error()


def test_u128_to_double_matches_python(tmp_path):
    """The statistics kernel's exact 128-bit -> float64 rounding, compiled for the host."""
    src = tmp_path / "t.cpp"
    src.write_text(
        '#include <cstdio>\n#include <cstdlib>\n#include "numerics.h"\n'
        "int main(int argc, char** argv) {\n"
        "  unsigned long long hi, lo;\n"
        "  while (scanf(\"%llx %llx\", &hi, &lo) == 2) {\n"
        "    unsigned __int128 v = ((unsigned __int128)hi << 64) | lo;\n"
        "    printf(\"%a\\n\", aa::u128_to_double_rn(v));\n  }\n  return 0;\n}\n")
    exe = tmp_path / "t"
    inc = os.path.join(ROOT, "paper_2101_00941_amd", "csrc")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", inc, str(src), "-o", str(exe)], check=True)
    rng = np.random.default_rng(1)
    vals = [0, 1, (1 << 53) - 1, 1 << 53, (1 << 53) + 1, (1 << 54) + 2, (1 << 54) + 6, (1 << 64) - 1,
            (1 << 64) + 2048 * 3, (1 << 127) + (1 << 74), (1 << 128) - 1]
    for bits in (54, 60, 70, 90, 110, 127):
        for _ in range(200):
            r = int.from_bytes(rng.bytes(16), "little") >> (128 - bits)
            vals.append(r | (1 << (bits - 1)))
    # exact halfway cases
    for sh in (1, 5, 30, 60):
        m = int(rng.integers(1 << 52, 1 << 53))
        vals.append((m << sh) | (1 << (sh - 1)))
    inp = "".join(f"{v >> 64:x} {v & ((1 << 64) - 1):x}\n" for v in vals)
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout.split()
    for v, s in zip(vals, out):
        assert float.fromhex(s) == float(v), v


def test_plan_rejects_bad_clipping():
    from paper_2101_00941_amd import AAError, Plan
    for c, it in ((-1.0, 2), (float("nan"), 1), (3.0, 17), (3.0, -1)):
        with pytest.raises(AAError):
            Plan(64, 20000, 1500.0, 1.5, 64e-6, np.arange(10.0), [1, 2], 6.0, clip_sigma=c, clip_iters=it,
                 host_only=True)
    Plan(64, 20000, 1500.0, 1.5, 64e-6, np.arange(10.0), [1, 2], 6.0, clip_sigma=3.0, clip_iters=16, host_only=True)


def test_plan_rejects_bad_boxcar_hierarchy():
    from paper_2101_00941_amd import AAError, Plan
    for w0 in (-1, 1):
        with pytest.raises(AAError):
            Plan(64, 20000, 1500.0, 1.5, 64e-6, np.arange(10.0), [2, 4], 6.0, boxcar_full_width=w0, host_only=True)
    Plan(64, 20000, 1500.0, 1.5, 64e-6, np.arange(10.0), [2, 4], 6.0, boxcar_full_width=2, host_only=True)


def test_plain_c_caller(tmp_path):
    """A C program (no Python) links the library and calls host-side entry points."""
    from paper_2101_00941_amd import _native
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = tmp_path / "abi_c"
    libdir = os.path.dirname(_native.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-O1", "-Wall", "-I", os.path.join(root, "include"),
                    os.path.join(root, "tests", "host", "abi_c_check.c"), "-L", libdir, "-l:libaa_mi355x.so",
                    f"-Wl,-rpath,{libdir}", "-o", str(exe), "-lm"], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr


def test_quad_variants_refuse_wide_residuals(aa):
    """Shifts within one quad of channels that differ by more than 1023 samples (10 MHz
    channels near 400 MHz, DM 100, 1 us sampling: about 4e5 samples): every quad
    shift-and-add variant refuses the plan with AA_EINVAL and says why, and the other
    kernel families still prepare their tables (host-only plan: tables only)."""
    from paper_2101_00941_amd import AAError, Plan
    p = Plan(8, 1 << 26, 400.0, 10.0, 1e-6, [0.0, 100.0], [1], 6.0, host_only=True)
    s = p.shifts().astype(np.int64)
    assert s[1, 3] - s[1, 0] > 1023
    variants = Plan.variants()
    quads = [v for v, i in enumerate(variants) if i["layout"] == 7]
    assert len(quads) >= 1
    for v in quads:
        with pytest.raises(AAError) as e:
            p.set_variant(v)
        assert e.value.code == aa.AA_EINVAL
        assert b"1023" in aa.lib().aa_last_error()
    for v in (1, 12, 20):
        p.set_variant(v)
        assert p.variant == v
