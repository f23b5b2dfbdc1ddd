"""The batched executor (include/fsd_batch.h) on the GPU: every problem's
result is bitwise the one of its own fsd_cn_step, whatever the lane count
(until the autotuner moves passes to other engines: then to the solver
tolerance); small float64 and mixed-precision members also match the
float64 oracle."""
import numpy as np
import pytest

import workloads
from oracle import cn, operators as op

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MEMBERS = [
    dict(dim=2, n=(127, 63), delta=(0.3, 0.6), kplus=(1, 1), kminus=(1, 1), M=8,
         solver="pcg", precision="fp64", tol=1e-10),
    dict(dim=2, n=(255, 31), delta=(0.7, 0.2), kplus=(1.5, 0.7), kminus=(0.6, 1.1), M=8,
         solver="gmres", precision="mixed", tol=1e-9),
    dict(dim=3, n=(31, 15, 63), delta=(0.3, 0.6, 0.8), kplus=(1, 2, 1), kminus=(2, 1, 1), M=8,
         solver="gmres", precision="fp64", tol=1e-10),
    dict(dim=3, n=(47, 47, 23), delta=(0.5, 0.4, 0.3), kplus=(1, 1, 1), kminus=(1, 1, 1), M=8,
         solver="pcg", precision="mixed", tol=1e-9),
    dict(dim=3, n=(15, 7, 15), delta=(0.2, 0.5, 0.9), kplus=(1, 1, 1), kminus=(1, 1, 1), M=4,
         solver="pcg", precision="fp64", tol=1e-12),
    dict(dim=2, n=(31, 15), delta=(0.4, 0.8), kplus=(1.2, 0.9), kminus=(0.5, 1.4), M=4,
         solver="gmres", precision="fp64", tol=1e-12),
]


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_21198_amd.batch import Batch
    from paper_2511_21198_amd.solver import Problem
    return Batch, Problem


def _inputs():
    us, Fs = [], []
    for i, kw in enumerate(MEMBERS):
        shape = tuple(reversed(kw["n"]))
        us.append(torch.from_numpy(workloads.random_grid(shape, 100 + i)).cuda())
        Fs.append(torch.from_numpy(workloads.random_grid(shape, 200 + i)).cuda())
    return us, Fs


def test_batch_bitwise_equals_single(mods):
    Batch, Problem = mods
    us, Fs = _inputs()
    ref = []
    for kw, u, F in zip(MEMBERS, us, Fs):
        p = Problem(**kw)
        a, _ = p.cn_step(u, F)
        b, _ = p.cn_step(a, F)
        ref.append(b.clone())
    for lanes in (1, 3, 4):
        bt = Batch(MEMBERS, streams=4)
        bt.set_lanes(lanes)
        o1, st1 = bt.cn_step(us, Fs)
        o2, st2 = bt.cn_step(o1, Fs)
        for i in range(len(MEMBERS)):
            assert torch.equal(o2[i], ref[i]), (lanes, i)
            assert st2[i]["converged"] == 1


def test_batch_autotune_then_step(mods):
    Batch, _ = mods
    us, Fs = _inputs()
    bt = Batch(MEMBERS, streams=4)
    ref, _ = bt.cn_step(us, Fs)
    ref = [r.clone() for r in ref]
    lanes, ms = bt.autotune(us, Fs)
    assert (lanes, bt.graphs) in ms and all(v > 0 for v in ms.values())
    out, _ = bt.cn_step(us, Fs)
    # the autotuner may move passes to other engines (tile shapes): the
    # operators then differ by rounding, and each step stops on the same
    # test, so the results agree to the solver tolerance
    for kw, a, b in zip(MEMBERS, out, ref):
        e = float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
        assert e <= 100 * kw["tol"], (e, kw)
    for i in range(len(MEMBERS)):
        assert "=" in bt.engines(i)


def test_batch_members_match_oracle(mods):
    Batch, _ = mods
    small = MEMBERS[4:]
    us, Fs = _inputs()
    us, Fs = us[4:], Fs[4:]
    bt = Batch(small, streams=2)
    u = us
    for _ in range(small[0]["M"]):
        u, st = bt.cn_step(u, Fs)
        u = [x.clone() for x in u]
    for kw, u0, F, ug in zip(small, us, Fs, u):
        orc = op.Problem(kw["dim"], list(kw["n"]), list(kw["delta"]), list(kw["kplus"]),
                         list(kw["kminus"]), T=1.0, M=kw["M"])
        ur, _ = cn.run(orc, u0.cpu().numpy(), lambda m: F.cpu().numpy(), tol=1e-13,
                       solver=kw["solver"])
        _close(ug.cpu().numpy(), ur, 1e-10)


def _close(a, b, bound):
    """Relative error in the 2-norm and in the max-norm (max |a-b| / max |b|)."""
    e2 = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    em = float(np.abs(a - b).max() / np.abs(b).max())
    assert e2 <= bound and em <= bound, (e2, em, bound)


# Mixed-precision members (the float32 inner solves inside float64 defect
# correction, PCG and left GMRES, 2D and 3D) solved tightly in a batch with a
# float64 member: each against the oracle's tightly solved steps, to the
# 1e-8 bound of the mixed-precision single-problem runs.
MIXED_MEMBERS = [
    dict(dim=2, n=(255, 31), delta=(0.7, 0.2), kplus=(1.5, 0.7), kminus=(0.6, 1.1), M=4,
         solver="gmres", precision="mixed", tol=1e-12, inner_tol=1e-5),
    dict(dim=3, n=(47, 47, 23), delta=(0.5, 0.4, 0.3), kplus=(1, 1, 1), kminus=(1, 1, 1), M=4,
         solver="pcg", precision="mixed", tol=1e-12, inner_tol=1e-5),
    dict(dim=3, n=(31, 15, 63), delta=(0.3, 0.6, 0.8), kplus=(1, 2, 1), kminus=(2, 1, 1), M=4,
         solver="gmres", precision="mixed", tol=1e-12, inner_tol=1e-3),
    dict(dim=2, n=(31, 15), delta=(0.4, 0.8), kplus=(1.2, 0.9), kminus=(0.5, 1.4), M=4,
         solver="gmres", precision="fp64", tol=1e-13),
]


def test_batch_mixed_members_match_oracle(mods):
    Batch, _ = mods
    us, Fs = [], []
    for i, kw in enumerate(MIXED_MEMBERS):
        shape = tuple(reversed(kw["n"]))
        us.append(torch.from_numpy(workloads.random_grid(shape, 400 + i)).cuda())
        Fs.append(torch.from_numpy(workloads.random_grid(shape, 500 + i)).cuda())
    bt = Batch(MIXED_MEMBERS, streams=2)
    u = us
    for _ in range(4):
        u, st = bt.cn_step(u, Fs)
        u = [x.clone() for x in u]
        assert all(s["converged"] == 1 for s in st)
    for kw, u0, F, ug in zip(MIXED_MEMBERS, us, Fs, u):
        orc = op.Problem(kw["dim"], list(kw["n"]), list(kw["delta"]), list(kw["kplus"]),
                         list(kw["kminus"]), T=1.0, M=kw["M"])
        ur, _ = cn.run(orc, u0.cpu().numpy(), lambda m: F.cpu().numpy(), tol=1e-13,
                       solver=kw["solver"])
        _close(ug.cpu().numpy(), ur, 1e-8 if kw["precision"] == "mixed" else 1e-10)


@pytest.mark.parametrize("kw", [MEMBERS[1], MEMBERS[3], MEMBERS[4], MEMBERS[5],
                                dict(MEMBERS[2], reorth_eta2=1.0),
                                dict(MEMBERS[2], solver="gmres2")],
                         ids=["gmres-mixed", "pcg-mixed", "pcg-fp64", "gmres-fp64",
                              "gmres-reorth", "gmres2"])
def test_graphs_bitwise_equal_direct(mods, kw):
    """Launch graphs of the Krylov chunks (fsd_set_graphs) replay the same
    kernels: five CN steps with graphs (every step replays the captured
    chunks several times, with the solver's own direct launches and host
    synchronisations in between) give bitwise the states of five steps
    with direct launches, step by step."""
    _, Problem = mods
    shape = tuple(reversed(kw["n"]))
    u0 = torch.from_numpy(workloads.random_grid(shape, 600)).cuda()
    F = torch.from_numpy(workloads.random_grid(shape, 601)).cuda()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        pd = Problem(**kw, stream=st)
        pg = Problem(**kw, stream=st)
        pg.set_graphs(True)
        ud, ug = u0.clone(), u0.clone()
        for m in range(5):
            ud, sd = pd.cn_step(ud, F)
            ug, sg = pg.cn_step(ug, F)
            st.synchronize()
            assert sd["iters"] == sg["iters"], (m, sd, sg)
            assert torch.equal(ud, ug), m
