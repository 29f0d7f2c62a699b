"""The vector-ALU issue-rate probe (amh_probe_valu) that the roofline's peak and instruction costs rest on: it
runs every instruction kind, and the rates keep the order the roofline assumes (a full-rate FMA issues at
least twice as fast as the reciprocal, and no kind beats the 2-clocks-per-wave-instruction ceiling)."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def amh():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_07920_amd as amh

    amh.lib()
    return amh


def test_probe_rates_are_ordered(amh):
    blocks, iters = 2048, 256
    winstr = 16.0 * iters * blocks * 4  # wave instructions per launch: 16 chains, 4 waves per workgroup
    ceiling = 256 * 4 * 2.4e9 / 2  # wave instructions per second at 2 clocks each on every SIMD
    rate = {}
    for kind, name in enumerate(amh.PROBE_KINDS):
        say(f"case probe kind {kind} ({name})")
        ms = min(amh.probe_valu(kind, blocks, iters) for _ in range(2))
        assert ms > 0.0
        rate[kind] = winstr / (ms / 1000.0)
        say(f"  {name}: {rate[kind] / ceiling:.3f} of the 2-clock ceiling")
        assert rate[kind] <= 1.05 * ceiling, name
    # v_fma_f32 with vector operands against v_rcp_f32 (quarter rate)
    assert rate[0] >= 2.0 * rate[2]
