"""The measurement probes behind the roofline peaks (ct_valu_probe,
ct_copy_probe): the copy moves every byte, the issue-rate probe writes
nothing, and both reject bad arguments."""
import pytest
import torch

pytestmark = pytest.mark.gpu

ct = pytest.importorskip("paper_1810_03275_amd")

DEV = torch.device("cuda")


def test_copy_probe_copies_exactly():
    print("copy probe", flush=True)
    g = torch.Generator(device="cpu").manual_seed(5)
    for n in (4, 1000, 1 << 20):          # fewer elements than threads, ragged, many strides
        src = torch.randn(n, generator=g).to(DEV)
        dst = torch.full_like(src, float("nan"))
        ct.copy_probe(src, dst, 64)
        torch.cuda.synchronize()
        assert torch.equal(src, dst)
    with pytest.raises(ValueError):
        ct.copy_probe(src, torch.empty(3, device=DEV), 64)
    with pytest.raises(ct.CtpdError):
        ct.copy_probe(src, dst, 0)


def test_valu_probe_runs_and_writes_nothing():
    print("valu probe", flush=True)
    out = torch.zeros(64, device=DEV)
    for kind, (_, per) in ct.VALU_PROBE_KINDS.items():
        assert ct.valu_probe(64, 256, out, kind) == 64 * 4 * 256 * 16 * per
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0
    with pytest.raises(ct.CtpdError):
        ct.valu_probe(64, 0, out)
    with pytest.raises(ValueError):
        ct.valu_probe(128, 16, out)      # out shorter than the grid
