"""The paper's synthetic sweeps (Sec. 6.1, 6.2) on the GPU against the oracle:
pat_psnr against the oracle's PSNR (Sec. 5.4), and one small detector curve
(every lambda of every method batched on each detector set) against the same
curve computed by the oracle from the same data."""
import math

import numpy as np
import pytest
import torch

import phantoms
from oracle import geometry as OG
from oracle import metrics as OM
from oracle import pdhg as OP

from gpu_common import oracle_problem

pytestmark = pytest.mark.gpu

pat = pytest.importorskip("paper_1707_02245_amd.pat")
EX = pytest.importorskip("paper_1707_02245_amd.experiments")


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [1, 257, 65536 + 17])
def test_psnr_matches_oracle(n, dt):
    rng = np.random.default_rng(n)
    gt = rng.uniform(0.0, 1.0, n)
    u = gt + 0.05 * rng.standard_normal(n)
    if dt == torch.float32:
        gt, u = gt.astype(np.float32).astype(np.float64), u.astype(np.float32).astype(np.float64)
    pp, ps = pat.psnr(torch.tensor(u, dtype=dt, device="cuda"), torch.tensor(gt, dtype=dt, device="cuda"))
    tol = 1e-12 if dt == torch.float64 else 1e-5
    assert pp == pytest.approx(OM.psnr_as_printed(u, gt), abs=tol * 100)
    assert ps == pytest.approx(OM.psnr(u, gt), abs=tol * 100)


def test_psnr_edge_cases():
    gt = torch.linspace(0.1, 1.0, 100, dtype=torch.float64, device="cuda")
    pp, ps = pat.psnr(gt.clone(), gt)
    assert math.isinf(pp) and pp > 0 and math.isinf(ps)
    with pytest.raises(pat.L.PatError) as e:
        pat.psnr(gt, -gt)
    assert e.value.status == pat.L.PAT_ERR_NUMERIC


def _oracle_data(desc, case, noise):
    n = desc["nx"]
    Af = OG.forward_matrix(OG.make_geometry(dict(desc, nx=2 * n, ny=2 * n)))
    fc = Af @ case["u_fine"].ravel()
    return fc + noise * np.linalg.norm(fc) / math.sqrt(fc.size) * case["noise"].ravel()[:fc.size]


def test_detector_curve_matches_oracle():
    """24^2 disc phantom, 16 and 64 detectors of the rotated array, TV and
    LS-T at three weights each, 150 iterations: every PSNR and the chosen
    weights against the oracle's reconstructions of the same data."""
    n, lams = 24, {"tv": (1e-3, 1e-2, 5e-2), "lst": (1e-3, 1e-2, 1e-1)}
    pts = EX.detector_curve(n=n, counts=(16, 64), family="disc", seed=3, methods=("tv", "lst"),
                            noise=0.02, data_fn=_oracle_data, lambdas=lams, iters=150)
    case = phantoms.make_case("disc", n, 3, 384, 2 * n)
    for pt in pts:
        desc = EX.sweep_geometry(n, pt["detectors"])
        A = OG.forward_matrix(OG.make_geometry(desc))
        f = _oracle_data(desc, case, 0.02)
        best = {}
        for row in pt["rows"]:
            kind = "tikhonov" if row["method"] == "lst" else row["method"]
            p = oracle_problem(A, f, n, kind, row["lam"])
            u = OP.pdhg_solve(p, OP.precond_diag(p), iters=150)["u"].reshape(n, n)
            want = OM.psnr_as_printed(u, case["u_gt"])
            print(f"{pt['detectors']} dets {row['method']} {row['lam']:.0e}: {row['psnr_printed']:.6f} "
                  f"oracle {want:.6f} dB", flush=True)
            assert row["psnr_printed"] == pytest.approx(want, abs=1e-8)
            assert row["psnr_standard"] == pytest.approx(OM.psnr(u, case["u_gt"]), abs=1e-8)
            if row["method"] not in best or want > best[row["method"]][1]:
                best[row["method"]] = (row["lam"], want)
        for m, (lam, _) in best.items():
            assert pt["best"][m]["lam"] == lam
