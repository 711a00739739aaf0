"""Build checks that need no GPU: every kernel of the last in-tree build of
librk (its compiler resource-usage record) keeps nothing on a per-lane stack
(no scratch, no dynamic stack, no vector registers spilled to memory), and
every scan kernel instantiation is present.  (Scalar registers spilled into
vector-register lanes use no memory and are allowed.)"""
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
USAGE = os.path.join(ROOT, "paper_1810_01051_amd", "_build", "resource_usage.json")


@pytest.fixture(scope="module")
def usage():
    if not os.path.exists(USAGE):
        pytest.skip("librk has not been built in this tree")
    return json.load(open(USAGE))


def test_no_kernel_uses_a_stack(usage):
    bad = {k: v for k, v in usage.items() if v.get("scratch", 0) or v.get("dyn_stack") or v.get("vgpr_spill", 0)}
    assert not bad, bad


def test_every_scan_instantiation_is_recorded(usage):
    scans = [k for k in usage if "scan_kernel" in k or "scan_list_kernel" in k]
    # 3 families x 4 geometries x 2 kernels
    assert len(scans) == 24, sorted(scans)
    assert any("paper_kernel" in k for k in usage)
