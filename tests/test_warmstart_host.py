"""Host-side logic of the warm-start driver (no GPU): the training
symmetries keep every (gradient, pressure) pair consistent, and the
network's parameter layout is what the layer calls assume."""

import torch


def test_symmetry_map_keeps_gradient_consistent_with_pressure():
    from paper_2311_16935_amd.warmstart import _symmetry

    n = 6
    z, y, x = torch.meshgrid(*(torch.arange(n, dtype=torch.float64),) * 3, indexing="ij")
    P = 0.3 * x * x + 0.7 * y * z - 0.2 * z + 0.5 * x * y + 0.1 * y * y
    g = torch.stack([0.6 * x + 0.5 * y, 0.7 * z + 0.5 * x + 0.2 * y, 0.7 * y - 0.2, torch.ones_like(x)], -1)
    gen = torch.Generator().manual_seed(0)
    for _ in range(24):
        X, T = _symmetry(g[None], P[None], gen)
        Pt, I = T[0], X[0, 1:-1, 1:-1, 1:-1]
        # central differences are exact for a quadratic pressure
        dx = (Pt[1:-1, 1:-1, 2:] - Pt[1:-1, 1:-1, :-2]) / 2
        dy = (Pt[1:-1, 2:, 1:-1] - Pt[1:-1, :-2, 1:-1]) / 2
        dz = (Pt[2:, 1:-1, 1:-1] - Pt[:-2, 1:-1, 1:-1]) / 2
        for k, d in enumerate((dx, dy, dz)):
            assert torch.allclose(I[..., k], d, atol=1e-12)
        assert torch.all(I[..., 3] == 1)


def test_parameter_layout():
    from paper_2311_16935_amd.warmstart import UNet

    layers, size = UNet.layout(32, 4, 4)
    names = list(layers)
    assert names[:2] == ["enc0a", "enc0b"] and names[-1] == "head"
    assert [layers[f"enc{l}b"].cout for l in range(4)] == [32, 64, 128, 256]
    total = sum(L.wsize + (L.cout if L.off_b >= 0 else 0) for L in layers.values())
    assert 5.5e6 < total < 5.7e6
    end = 0
    for L in layers.values():
        # 128-byte aligned BF16 slices (16-byte vector loads), no overlap
        assert L.off_w % 64 == 0 and L.off_w >= end
        end = L.off_w + L.wsize
        if L.off_b >= 0:
            assert L.off_b % 64 == 0 and L.off_b >= end
            end = L.off_b + L.cout
        assert L.kind == "head" or L.cout % 8 == 0
    assert end <= size
    assert layers["up0"].off_b < 0 and layers["up0"].taps == 8 and layers["dec0a"].cin == 64
