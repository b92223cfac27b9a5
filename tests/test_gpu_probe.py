"""The device-ceiling probes run, keep their work (the instruction counts
the profiles rely on are those of the loops), and report a plausible clock."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", [1, 2])
def test_probe_runs_and_clocks(kind):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_04090_amd import vsfe
    blocks = 64
    sink = torch.full((blocks * 256,), 7, dtype=torch.int32, device="cuda")
    clocks = torch.zeros(2, dtype=torch.int64, device="cuda")
    vsfe.probe(kind, blocks, 200, sink, clocks)
    torch.cuda.synchronize()
    cyc, wall = clocks.cpu().tolist()
    assert cyc > 0 and wall > 0
    ghz = cyc / (wall / 100e6) / 1e9
    assert 0.5 < ghz < 3.5, ghz
    # the sink is written only in a case that cannot occur
    assert (sink == 7).all()
