"""The 16x16-tile FP32 encoder's launch forms against each other and the FP64 reference.

The encoder's stage-1 Im rows read a second LDS table holding i * d when both tables fit a
CU's LDS; a launch with at least 8 tiles of 16 patches per CU then runs 8-wave blocks (one
per CU), a smaller one 4-wave blocks.  A dictionary too large for both tables (M = 200 at
15x15, 2 x 84 KB) takes the other form, whose Im rows negate what they read from d.  Every
patch is coded on its own, so one launch over all patches and launches over chunks of 1,600
patches (100 tiles) must give the same codes bit for bit.
The one-launch codes are also held to the parity bar against the FP64 reference on their
first patches (selected (atom, angle) sets equal on >= 99.9%, every matched coefficient
within 1e-4 relative).  The cases cover both grids and both annular bases, one to eight
16-row angle tiles (even R split by parity, odd R direct) and K from 2 to 8.
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
CHUNK = 1600
N_REF = 1200

# (id, basis kind, N, S, T, M, R, K)
CASES = [
    ("grid15-ragged-config", "grid", 15, 7, 7, 128, 64, 6),
    ("grid11-K8-oddR", "grid", 11, 5, 5, 40, 33, 8),
    ("grid11-R32", "grid", 11, 5, 5, 64, 32, 2),
    ("grid11-R128", "grid", 11, 5, 5, 24, 128, 3),       # four 16-row angle tiles after the split
    ("grid11-R97", "grid", 11, 5, 5, 16, 97, 2),         # odd R: eight tiles of the direct DFT
    ("grid15-R100-K8", "grid", 15, 7, 7, 32, 100, 8),
    ("annular11", "annular", 11, 0, 0, 64, 64, 4),
    ("annular15", "annular", 15, 0, 0, 48, 30, 2),
    ("grid15-large-dictionary", "grid", 15, 7, 7, 200, 16, 2),
]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_04374_amd import rsc
    rsc.lib()
    return torch.device("cuda:0")


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_one_launch_equals_chunks_and_reference(dev, case):
    from paper_1806_04374_amd import rsc
    name, kind, N, S, T, M, R, K = case
    if kind == "annular":
        basis = orc.build_annular_basis(N)
        h = rsc.rsc_create_annular(N)
    else:
        basis = orc.build_basis(N, S, T)
        h = rsc.rsc_create(N, S, T)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    P = 8 * n_cu * 16 + 777                    # enough tiles for the i * d form, ragged last tile
    seed = 300 + CASES.index(case)
    D = wl.draw_dictionary(M, basis.B, seed=seed)
    rsc.rsc_set_dictionary(h, D.astype(np.float32), R)
    rsc.rsc_set_tile(h, "16")
    d = wl.draw_mixtures(P, N, M, min(3, M), 0.02, seed=seed)
    X = orc.synthesize(basis, D, d.atom, d.angle, d.weight, d.noise).astype(np.float32)
    print("case", name, "P", P, flush=True)
    xh = rsc.rsc_project(h, torch.from_numpy(X).to(dev))
    one = [t.cpu().numpy() for t in rsc.rsc_omp_encode(h, xh, K)]
    parts = [[t.cpu().numpy() for t in rsc.rsc_omp_encode(h, xh[i:i + CHUNK].contiguous(), K)]
             for i in range(0, P, CHUNK)]
    torch.cuda.synchronize()
    for j, label in enumerate(["atom", "angle", "coef", "resid2"]):
        whole = np.concatenate([p[j] for p in parts])
        assert np.array_equal(one[j], whole), (name, label, int((one[j] != whole).sum()))
    xh_ref, code = orc.encode(basis, D, R, X[:N_REF].astype(np.float64), K)
    rep = compare_codes(one[0][:N_REF], one[1][:N_REF], one[2][:N_REF], code, COEF_REL,
                        xnorm=np.linalg.norm(xh_ref, axis=1))
    print(name, rep, flush=True)
    assert rep.match_rate >= MATCH, (name, str(rep))
    assert rep.coef_bad == 0, (name, str(rep))
    h.close()
