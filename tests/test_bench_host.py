"""Host-side logic of bench.py (no GPU): the one-GPU contract, the DOF-update counts the throughput
is quoted in, the time-to-tolerance reading of a residual history, and the guard that attaches a
committed counter summary's traffic only while the kernel sources are the ones it was taken with."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr


@pytest.mark.parametrize("ne,plev,nsm,nv,dim,expect", [
    (64, (2, 1, 0), (5, 10, 20), 4, 2, 4.9e4),                  # config 1
    (4096, (3, 2, 1), (5, 10, 20), 4, 2, 6.9e6),                # config 2
    (8192, (4, 2, 1), (5, 10, 20), 4, 2, 1.7e7),                # config 3
    (8192, (4, 3, 2, 1, 0), (5, 10, 20, 20, 20), 4, 2, 3.6e7),  # config 3'
    (36864, (2, 1, 0), (5, 10, 20), 5, 3, 8.3e7),               # config 5, P{2-1-0}
    (36864, (3, 2, 1, 0), (5, 10, 20, 20), 5, 3, 2.8e8),        # config 5, P{3-2-1-0}
])
def test_dof_updates_per_vcycle(ne, plev, nsm, nv, dim, expect):
    """Pre- and post-smoothing on every level but the coarsest, which smooths once; the survey's
    table of the configurations gives the counts to two digits."""
    got = bench.dof_updates_per_vcycle(ne, plev, nsm, nv=nv, dim=dim)
    assert abs(got - expect) <= 0.05 * expect, (got, expect)
    # written out for the headline: 10 sweeps of 64 points, 20 of 27, 40 of 8, 20 of 1 per element
    if plev == (3, 2, 1, 0) and dim == 3:
        assert got == 36864 * 5 * (10 * 64 + 20 * 27 + 40 * 8 + 20 * 1)


def test_time_to_tolerances_reads_the_first_crossing():
    hist = [1.0, 1e-2, 5e-5, 2e-5, 5e-7, 2e-9, 3e-9]         # 6 V-cycles in 0.6 s: 0.1 s each
    out, floors = bench.time_to_tolerances([{"history": hist, "seconds": 0.6, "n_vcycles": 6}])
    assert out["1e-04"] == [pytest.approx(0.2)]
    assert out["1e-06"] == [pytest.approx(0.4)]
    assert out["1e-08"] == [pytest.approx(0.5)]
    assert floors == [pytest.approx(2e-9)]
    out, _ = bench.time_to_tolerances([{"history": [1.0, 0.5], "seconds": 0.1, "n_vcycles": 1}])
    assert out["1e-04"] == [None]


def test_measured_traffic_requires_the_current_sources(tmp_path):
    good = tmp_path / "good.txt"
    good.write_text("# header\ntraffic_bytes_per_launch: 12345\n"
                    f"kernel_source_hash: {bench.kernel_source_hash(bench.KERNEL_SOURCES_3D)}\n")
    assert bench.measured_traffic(str(good), bench.KERNEL_SOURCES_3D) == 12345.0
    stale = tmp_path / "stale.txt"
    stale.write_text("traffic_bytes_per_launch: 12345\nkernel_source_hash: 0000000000000000\n")
    assert bench.measured_traffic(str(stale), bench.KERNEL_SOURCES_3D) is None
    assert bench.measured_traffic(str(tmp_path / "missing.txt"), bench.KERNEL_SOURCES_3D) is None


def test_committed_headline_profile_matches_the_sources():
    """The roofline's traffic figure comes from this summary; it must describe the current kernels."""
    t = bench.measured_traffic(bench.PROFILE_PMC_SPHERE3, bench.KERNEL_SOURCES_3D)
    assert t is not None
    alg = 36864 * 320 * (4 * 320 + 24)                       # Ne n (4 npad + 24) B, npad = n = 320
    assert alg <= t <= 1.2 * alg


def test_kernel_hash_covers_the_sweep_sources():
    hdr = open(os.path.join(ROOT, "paper_1908_03972_amd", "csrc", "fr3_kernels.hip")).read()
    for inc in ("internal.hpp", "hex_points.hpp", "physics3.hpp", "block_loads.hpp"):
        if f'#include "{inc}"' in hdr:
            assert inc in bench.KERNEL_SOURCES_3D, inc
    hdr2 = open(os.path.join(ROOT, "paper_1908_03972_amd", "csrc", "fr_kernels.hip")).read()
    for inc in ("internal.hpp", "vcycle.hpp", "block_loads.hpp"):
        if f'#include "{inc}"' in hdr2:
            assert inc in bench.KERNEL_SOURCES_2D, inc
