"""Register use of the transform kernels on the bench's paths (CPU: compiles
the gfx950 code with the compiler's resource remarks, no GPU needed).

The kernels keep their occupancy only while the compiler does not hold one
transform's index arithmetic, a sunk sum or the tile's load addresses across
another transform; a source change that brings such a pattern back shows up
here as spilled registers or fewer waves per SIMD before it shows up as time.
"""

import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_2103_03658_amd import build

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None and
                                not os.path.exists("/opt/rocm/bin/hipcc"),
                                reason="hipcc not available")

# demangled kernel -> minimum waves per SIMD (and no spilled VGPRs)
EXPECT_F64 = {
    "fl::k_mid<double, 1024, 16>": 3,
    "fl::k_first<double, 1024, 8>": 4,
    "fl::k_last<double, 1024, 8>": 4,
    "fl::k_sine_cols<double, 1024, 8, true, true, false>": 4,
    "fl::k_sine_cols<double, 1024, 8, false, false, true>": 5,
    "fl::k_sine_cols<double, 1024, 8, false, false, false>": 5,
    "fl::k_sine_mid<double, 1024, 16>": 3,
    "fl::k_sine_mid<double, 1024, 8>": 4,
    "fl::k_mid<double, 2048, 16>": 3,
}
EXPECT_F32 = {
    "fl::k_mid<float, 1024, 16>": 5,
    "fl::k_sine_mid<float, 1024, 16>": 5,
    "fl::k_sine_cols<float, 1024, 8, true, true, false>": 4,
    "fl::k_sine_cols<float, 1024, 16, true, true, false>": 4,
    "fl::k_sine_cols<float, 1024, 16, false, false, true>": 5,
    "fl::k_first<float, 2048, 16>": 4,
    "fl::k_mid<float, 2048, 16>": 4,
    "fl::k_last<float, 2048, 16>": 4,
}


def _instantiation_unit():
    """A translation unit that instantiates only the kernels checked here,
    from the same header and flags as the library (a fraction of its
    compile time)."""
    lines = ['#include "passes_impl.h"', "namespace fl {"]
    for name in list(EXPECT_F64) + list(EXPECT_F32):
        kern = name.split("<", 1)[0].replace("fl::", "")
        targs = name[name.index("<"):]
        t = "double" if "<double" in name else "float"
        arg = {"k_mid": "MidArgs", "k_first": "FirstArgs", "k_last": "LastArgs",
               "k_sine_cols": "SineArgs", "k_sine_mid": "SineMidArgs"}[kern]
        lines.append(f"template __global__ void {kern}{targs}({arg}<{t}>);")
    lines.append("}")
    return "\n".join(lines) + "\n"


def _resources():
    """Demangled kernel name -> dict(vgpr, spill, waves) from the remarks."""
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "kernels.hip")
        with open(src, "w") as fh:
            fh.write(_instantiation_unit())
        cmd = [build.hipcc()] + build.FLAGS + [
            "-c", src, "-o", os.path.join(td, "k.o"), "-Rpass-analysis=kernel-resource-usage"]
        res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    out, cur = {}, None
    for line in res.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            out[cur] = {}
            continue
        if cur is None:
            continue
        for key, pat in (("vgpr", r"\bVGPRs: (\d+)"), ("spill", r"VGPRs Spill: (\d+)"),
                         ("waves", r"Occupancy \[waves/SIMD\]: (\d+)")):
            m = re.search(pat, line)
            if m:
                out[cur][key] = int(m.group(1))
    names = list(out)
    dm = subprocess.run(["c++filt"], input="\n".join(names), capture_output=True,
                        text=True).stdout.splitlines()
    return {d.split("(")[0].replace("void ", "", 1): out[n] for n, d in zip(names, dm)}


@pytest.fixture(scope="module")
def resources():
    if shutil.which("c++filt") is None:
        pytest.skip("c++filt not available")
    return _resources()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_bench_kernels_keep_their_waves_without_spills(resources, prec):
    got = resources
    expect = EXPECT_F64 if prec == "f64" else EXPECT_F32
    bad = []
    for name, waves in expect.items():
        assert name in got, f"{name} not instantiated"
        r = got[name]
        if r.get("spill", 0) != 0 or r.get("waves", 0) < waves:
            bad.append(f"{name}: {r} (want >= {waves} waves, no spills)")
    assert not bad, "\n".join(bad)
