"""The allocation-free template entry point (lpp_template_plain_noalloc)
through the C ABI against the allocating one (lpp_template_plain): two calls
in a row on one device, the second with fewer points, host and device I/O.
Both run the same kernels per parameter point, so the outputs agree to the
FP64 parity bar (here they are expected to be the same bits)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _tables():
    k = np.exp(np.linspace(np.log(1e-5), np.log(1e3), 4096))
    pfid = 2e4 * (k / 0.02) / (1 + (k / 0.02) ** 2) ** 1.4
    r_q = np.linspace(4.0, 2500.0, 250)
    Q = np.vstack([np.exp(-r_q / 800.0) * (1.0 if i == 0 else 0.25 * (-1) ** i / (i + 1)) *
                   (1 + 0.1 * np.cos(r_q / 200.0 + i)) for i in range(5)])
    return pfid, r_q, Q


def test_template_noalloc_matches_allocating_entry_point():
    import torch
    import paper_2202_11839_amd as lpp
    from synth import EMU_RANGES, latin_hypercube
    assert torch.cuda.is_available()
    lpp.load()
    pfid, r_q, Q = _tables()
    kout = np.arange(1, 31) * 0.01
    # call 1: 300 points (three passes through the static scratch, the last ragged), host I/O
    pts = latin_hypercube(300, EMU_RANGES, seed=21)
    want = lpp.template_plain(pfid, 1e-5, 1e3, r_q, Q, pts, kout, 1.4e-3, 0.2)
    got = lpp.template_plain_noalloc(pfid, 1e-5, 1e3, r_q, Q, pts, kout, 1.4e-3, 0.2)
    scale = np.max(np.abs(want), axis=(0, 2))
    err = np.max(np.abs(got - want), axis=(0, 2)) / scale
    assert np.all(err <= 1e-12), err
    # call 2: 40 points, device I/O, other tables (the scratch keeps call 1's contents)
    pts2 = latin_hypercube(40, EMU_RANGES, seed=22)
    Q2 = Q * np.array([[1.0], [0.5], [2.0], [1.0], [0.0]])
    kout2 = np.linspace(0.005, 0.4, 57)
    P = torch.tensor(pts2, dtype=torch.float64, device="cuda")
    want2 = torch.zeros((40, 5, 57), dtype=torch.float64, device="cuda")
    got2 = torch.full((40, 5, 57), np.nan, dtype=torch.float64, device="cuda")
    lpp.template_plain(pfid, 1e-5, 1e3, r_q, Q2, P, kout2, 2.0e-3, 0.25, out=want2)
    lpp.template_plain_noalloc(pfid, 1e-5, 1e3, r_q, Q2, P, kout2, 2.0e-3, 0.25, out=got2)
    w2, g2 = want2.cpu().numpy(), got2.cpu().numpy()
    assert np.all(np.isfinite(g2))
    err2 = np.max(np.abs(g2 - w2), axis=(0, 2)) / np.max(np.abs(w2), axis=(0, 2))
    assert np.all(err2 <= 1e-12), err2
    print(f"\nnoalloc vs allocating: max rel diff {max(err.max(), err2.max()):.1e}, "
          f"bitwise equal: {np.array_equal(got, want) and np.array_equal(g2, w2)}")


def test_template_noalloc_rejects_bad_arguments():
    import paper_2202_11839_amd as lpp
    pfid, r_q, Q = _tables()
    pts = np.array([[0.02, 1.5, 0.7, 0.8, 1.0]])
    with pytest.raises(lpp.LppError) as e:
        lpp.template_plain_noalloc(pfid, 1e-5, 1e3, r_q, Q, pts, np.linspace(0.01, 0.3, 300), 1.4e-3, 0.2)
    assert e.value.status == 1   # n_k above 256
    with pytest.raises(lpp.LppError) as e:
        lpp.template_plain_noalloc(pfid, 1e-5, 1e3, r_q[::-1].copy(), Q, pts, np.array([0.1]), 1.4e-3, 0.2)
    assert e.value.status == 1   # r_q not increasing
