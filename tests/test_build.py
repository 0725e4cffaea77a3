"""The gfx950 kernels compile with no scratch memory and no register spills
(a private segment in a layer kernel means operands round-trip through
memory and the MFMA pipes starve).  CPU only: cross-compiles with hipcc."""

import shutil

import pytest

from paper_2107_02737_amd.build import hipcc, kernel_resources


@pytest.fixture(scope="module")
def resources():
    try:
        hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    return kernel_resources()


def test_every_kernel_present(resources):
    names = " ".join(resources)
    for k in ["k_gershgorin_rows", "k_bounds_final", "k_input_layer", "k_split", "k_sym_split",
              "k_sym_f32", "k_finish_loop"]:
        assert k in names


def test_no_scratch_no_spills(resources):
    for name, r in resources.items():
        assert r["private_segment_fixed_size"] == 0, name
        assert r["vgpr_spill_count"] == 0, name


def test_layer_kernels_fit_their_occupancy(resources):
    for name, r in resources.items():
        if "k_sym" in name:
            assert r["vgpr_count"] <= 256, name          # two waves per SIMD
            assert r["group_segment_fixed_size"] <= 160 * 1024, name


def test_hipcc_on_path_or_rocm():
    assert shutil.which("hipcc") or hipcc()
