"""GPU tests of fem_set_allocator: handle memory drawn from a caller's allocator (torch's
caching allocator, or a counting one) gives the same pattern and the same sums as
hipMalloc'd handles; every buffer comes back through the allocator it was drawn from;
an allocator that returns NULL makes the build fail with FEM_ERR_OOM and release what it
had drawn."""

import numpy as np
import pytest

import meshgen
import oracle
from tests._util import scaled_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-12


def fem():
    import paper_1802_03433_amd as F

    return F


@pytest.fixture(autouse=True)
def default_allocator_after():
    yield
    fem().set_allocator()


def _dev(m):
    F = fem()
    dev = torch.device("cuda:0")
    return F.Mesh(torch.from_numpy(m.coords).to(dev), torch.from_numpy(m.conn).to(dev), m.order)


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


class Counting:
    """Draws from torch's caching allocator and records what is live."""

    def __init__(self, fail_after=None):
        self.live = {}
        self.calls = 0
        self.fail_after = fail_after
        self.bad_release = 0

    def alloc(self, n):
        self.calls += 1
        if self.fail_after is not None and self.calls > self.fail_after:
            return 0
        p = torch.cuda.caching_allocator_alloc(n, torch.cuda.current_device())
        self.live[p] = n
        return p

    def release(self, p):
        if p not in self.live:
            self.bad_release += 1
            return
        del self.live[p]
        torch.cuda.caching_allocator_delete(p)


def test_torch_allocator_same_results_and_accounting():
    F = fem()
    m = meshgen.cube_tet(12, seed=15)  # 10368 elements: several tiles and a ragged one
    d = _dev(m)
    kap_np = meshgen.coefficients(m.n_elems, "helmholtz", seed=3)
    kap = torch.from_numpy(kap_np).cuda()
    form = F.Form("helmholtz", "sinprod")
    ref = F.Pattern(d)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    F.use_torch_allocator()
    pat = F.Pattern(d)
    F.set_allocator()
    torch.cuda.synchronize()
    grown = torch.cuda.memory_allocated() - before
    assert grown >= pat.device_bytes > 0
    assert pat.device_bytes == ref.device_bytes
    for a, b in zip(ref.export(), pat.export()):
        assert np.array_equal(_np(a), _np(b))
    assert np.array_equal(_np(ref.colours()), _np(pat.colours()))
    rp, ci = oracle.pattern(4, 1, m.n_nodes, m.conn)
    ov, orhs, oav, oar = oracle.assemble_p1(m, kap_np[0], 1.0, "sinprod", None, rp, ci)
    for scatter in ("atomic", "coloured", "two-pass"):
        v, r = F.assemble(pat, d, form, kap, scatter=scatter)
        ok, worst = scaled_close(_np(v), ov, oav, RTOL)
        assert ok, (scatter, worst)
        ok, worst = scaled_close(_np(r), orhs, oar, RTOL)
        assert ok, (scatter, worst)
        if scatter != "atomic":
            v0, r0 = F.assemble(ref, d, form, kap, scatter=scatter)
            assert np.array_equal(_np(v), _np(v0)) and np.array_equal(_np(r), _np(r0))
    del v, r, v0, r0
    torch.cuda.synchronize()
    # the two-pass partial sums were drawn at the first two-pass call, under the default
    mid = torch.cuda.memory_allocated()
    pat.close()
    assert mid - torch.cuda.memory_allocated() == grown


def test_every_buffer_released_through_its_own_allocator():
    F = fem()
    a = Counting()
    F.set_allocator(a.alloc, a.release)
    m1 = meshgen.cube_tet(6, seed=2)
    m2 = meshgen.cube_tet(2, 2, seed=4)
    d1, d2 = _dev(m1), _dev(m2)
    pat = F.Pattern(d1)
    batch = F.Batch([d1, d2, _dev(meshgen.square_tri(5, seed=6))])
    assert all(p % 256 == 0 for p in a.live)
    assert sum(a.live.values()) == pat.device_bytes + batch.device_bytes
    # a two-pass call draws the partial sums lazily, from the allocator now registered
    b = Counting()
    F.set_allocator(b.alloc, b.release)
    kap = torch.from_numpy(meshgen.coefficients(m1.n_elems, "helmholtz", seed=1)).cuda()
    F.assemble(pat, d1, F.Form("helmholtz", "sinprod"), kap, scatter="two-pass")
    torch.cuda.synchronize()
    assert b.live and all(p % 256 == 0 for p in b.live)
    n_b = len(b.live)
    F.set_allocator()
    other = F.Pattern(d2, ncomp=3)  # hipMalloc: neither counter moves
    assert len(b.live) == n_b and a.calls == len(a.live)
    pat.close()
    assert not b.live
    batch.close()
    other.close()
    assert not a.live and a.bad_release == 0 and b.bad_release == 0


@pytest.mark.parametrize("fail_after", [0, 1, 4, 12])
def test_allocator_null_is_oom_and_releases(fail_after):
    F = fem()
    a = Counting(fail_after)
    F.set_allocator(a.alloc, a.release)
    m = meshgen.cube_tet(4, seed=5)
    d = _dev(m)
    with pytest.raises(F.FemError) as e:
        F.Pattern(d)
    assert e.value.code == -3 and "NULL" in str(e.value)
    assert a.calls == fail_after + 1
    assert not a.live and a.bad_release == 0
    with pytest.raises(F.FemError) as e:
        F.Batch([d, _dev(meshgen.cube_tet(1, 2, seed=1))])
    assert e.value.code == -3
    assert not a.live and a.bad_release == 0
    F.set_allocator()
    F.Pattern(d).close()  # the default works again
