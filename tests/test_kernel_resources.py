"""Register, spill and workgroup-memory budgets of the MHD stage kernels, read from the
compiler's resource report for gfx950 (host only: hipcc cross-compiles, no GPU needed).

These are performance assumptions of the kernel design, not correctness: the FP64 PPM +
HLLD flux/update kernel runs three waves per SIMD (three workgroups' memory within the
CU's 160 KiB) with at most a few loop-invariant dwords spilled, every FP32 flux/update
kernel four, the FP64 HLLE and donor-cell ones three, the FP64 time-step CT kernel
three, and no other MHD stage kernel spills.  A different compiler can move them without changing any result; a
failure names the budget that moved.
"""
import re
import subprocess

import pytest

from paper_2608_14048_amd import build as B

LDS_PER_CU = 160 * 1024


def _resources(source: str) -> dict:
    flags = [f for f in B.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    cmd = [B.hipcc(), *flags, "-c", "--offload-device-only", "-o", "/dev/null",
           f"{B.CSRC}/{source}", "-Rpass-analysis=kernel-resource-usage"]
    try:
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    except FileNotFoundError:
        pytest.skip("hipcc not found")
    assert r.returncode == 0, r.stderr[-2000:]
    out, cur = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[[^\]]*\])?: (\d+) \[-Rpass", line)
        if m and cur is not None:
            cur[m.group(1)] = int(m.group(2))
    return out


@pytest.fixture(scope="module")
def fused():
    return _resources("mhd_fused.hip")


def _one(res: dict, prefix: str) -> dict:
    hits = [v for k, v in res.items() if k.startswith(prefix)]
    assert len(hits) == 1, (prefix, sorted(res))
    return hits[0]


# mangled names: k_flux3<RECON, RS, IN, real>, k_ct_update<CFL, IN, real, rows>
FLUX_PPM_HLLD_F64 = ("_ZN3mhd7k_flux3ILi2ELi1ELb0EdE", "_ZN3mhd7k_flux3ILi2ELi1ELb1EdE")
CT_CFL_F64 = "_ZN3mhd11k_ct_updateILb1ELb0EdLi4EE"


@pytest.mark.parametrize("name", FLUX_PPM_HLLD_F64)
def test_fp64_ppm_flux_kernel_runs_three_waves(fused, name):
    k = _one(fused, name)
    assert k["VGPRs"] + k.get("AGPRs", 0) <= 168, k
    assert 3 * k["LDS Size"] <= LDS_PER_CU, k
    assert k["Occupancy"] >= 3, k
    # a few loop-invariant values reloaded once per plane (measured 24 bytes per lane)
    assert k["ScratchSize"] <= 32, k


def test_fp64_time_step_ct_kernel_runs_three_waves(fused):
    k = _one(fused, CT_CFL_F64)
    assert k["Occupancy"] >= 3, k
    assert k["ScratchSize"] == 0, k


def test_fp32_flux_kernels_run_four_waves_and_fp64_hlle_three(fused):
    flux = {n: k for n, k in fused.items() if n.startswith("_ZN3mhd7k_flux3I")}
    assert len(flux) == 24, sorted(flux)
    for n, k in flux.items():
        # mangled template arguments: <RECON, RS, IN, real>
        m = re.match(r"_ZN3mhd7k_flux3ILi(\d)ELi(\d)ELb\dE([df])E", n)
        recon, rs, real = int(m.group(1)), int(m.group(2)), m.group(3)
        if real == "f":
            assert k["Occupancy"] >= 4, (n, k)
        elif rs == 0 or recon == 0:
            assert k["Occupancy"] >= 3, (n, k)


def test_other_stage_kernels_do_not_spill(fused):
    stage = {n: k for n, k in fused.items()
             if ("k_flux3" in n or "k_ct_update" in n) and not n.startswith(FLUX_PPM_HLLD_F64)}
    assert len(stage) >= 20, sorted(fused)
    spills = {n: k["ScratchSize"] for n, k in stage.items() if k["ScratchSize"]}
    assert not spills, spills
