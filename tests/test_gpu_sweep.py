"""A seeded sweep over the encoder's configuration space against the FP64 reference.

Forty cases drawn once from a fixed seed, each a few hundred patches of mixtures of
rotated atoms plus noise (the generator of the scale workload), spread over every path
of rsc_omp_encode: the grid of profiles at N = 11 (auto, 16x16 and 32x32 tiles), N = 13
(the same S = T = 5 encoder on another disk) and N = 15, the BF16 and FP16 forms, and the
paper's annular basis at N = 11 and 15; atom counts from 1 to 128, R from 1 to 128 (even
and odd; 16-bit forms R <= 64, annular and 32x32 tiles even R <= 64), K from 1 to the
path's limit, patch counts that leave a ragged last tile.

Acceptance as for the other parity tests: selected (atom, angle) sets equal on >= 99.9% of
patches, every coefficient of a matched patch within 1e-4 (relative, with the floor of
tests/parity.py), and the reported residual norms within 1e-3 relative (+1e-5 ||x||^2).
"""
import numpy as np
import pytest

from oracle import rsc_oracle as orc
from paper_1806_04374_amd import workloads as wl
from tests.parity import compare_codes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MATCH = 0.999
COEF_REL = 1e-4

# family: (basis kind, N, S, T, precision, tile, M max, R choice, K max)
FAMILIES = [
    ("grid", 11, 5, 5, "fp32", "auto", 128, "any128", 8),
    ("grid", 11, 5, 5, "fp32", "32", 128, "even64", 4),
    ("grid", 11, 5, 5, "fp32", "16", 128, "any128", 8),
    ("grid", 13, 5, 5, "fp32", "auto", 128, "any128", 8),
    ("grid", 15, 7, 7, "fp32", "auto", 128, "any96", 8),
    ("grid", 11, 5, 5, "bf16", "auto", 128, "any64", 8),
    ("grid", 11, 5, 5, "fp16", "auto", 128, "any64", 8),
    ("grid", 15, 7, 7, "bf16", "auto", 128, "any64", 8),
    ("annular", 11, 0, 0, "fp32", "auto", 64, "even64", 4),
    ("annular", 15, 0, 0, "fp32", "auto", 48, "even64", 4),
]


def _cases():
    rng = np.random.default_rng(20180612)
    out = []
    for i in range(40):
        kind, N, S, T, prec, tile, mmax, rch, kmax = FAMILIES[i % len(FAMILIES)]
        M = int(rng.integers(1, mmax + 1))
        if rch == "any128":
            R = int(rng.integers(1, 129))
        elif rch == "any96":
            R = int(rng.integers(1, 97))
        elif rch == "any64":
            R = int(rng.integers(1, 65))
        else:
            R = 2 * int(rng.integers(1, 33))
        K = int(rng.integers(1, kmax + 1))
        P = int(rng.integers(300, 701))
        out.append(dict(i=i, kind=kind, N=N, S=S, T=T, prec=prec, tile=tile, M=M, R=R, K=K, P=P))
    return out


CASES = _cases()


def _id(c):
    geo = f"ann{c['N']}" if c["kind"] == "annular" else f"g{c['N']}"
    return f"{c['i']:02d}-{geo}-{c['prec']}-t{c['tile']}-M{c['M']}-R{c['R']}-K{c['K']}-P{c['P']}"


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_04374_amd import rsc
    rsc.lib()
    return torch.device("cuda:0")


@pytest.mark.parametrize("c", CASES, ids=[_id(c) for c in CASES])
def test_sweep_case(dev, c):
    from paper_1806_04374_amd import rsc
    if c["kind"] == "annular":
        basis = orc.build_annular_basis(c["N"])
        h = rsc.rsc_create_annular(c["N"])
    else:
        basis = orc.build_basis(c["N"], c["S"], c["T"])
        h = rsc.rsc_create(c["N"], c["S"], c["T"], prec=c["prec"])
    seed = 1000 + c["i"]
    D = wl.draw_dictionary(c["M"], basis.B, seed=seed)
    rsc.rsc_set_dictionary(h, D.astype(np.float32), c["R"])
    if c["tile"] != "auto":
        rsc.rsc_set_tile(h, c["tile"])
    d = wl.draw_mixtures(c["P"], c["N"], c["M"], min(3, c["M"]), 0.02, seed=seed)
    X = orc.synthesize(basis, D, d.atom, d.angle, d.weight, d.noise).astype(np.float32)
    print("case", _id(c), flush=True)
    xh = rsc.rsc_project(h, torch.from_numpy(X).to(dev))
    atom, angle, coef, r2 = rsc.rsc_omp_encode(h, xh, c["K"])
    torch.cuda.synchronize()
    xh_ref, code = orc.encode(basis, D, c["R"], X.astype(np.float64), c["K"])
    rep = compare_codes(atom.cpu().numpy(), angle.cpu().numpy(), coef.cpu().numpy(), code, COEF_REL,
                        xnorm=np.linalg.norm(xh_ref, axis=1))
    print(_id(c), rep, flush=True)
    assert rep.match_rate >= MATCH, str(rep)
    assert rep.coef_bad == 0, str(rep)
    r2 = r2.cpu().numpy()
    close = np.abs(r2 - code.resid2) <= 1e-3 * code.resid2 + 1e-5 * np.einsum("ij,ij->i", xh_ref, xh_ref) + 1e-12
    assert close.mean() >= MATCH, close.mean()
    h.close()
