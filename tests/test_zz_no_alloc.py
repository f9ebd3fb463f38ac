"""tlfea_internal_force_noalloc through the C ABI: bitwise the forward of
tlfea_internal_force, on two calls in a row (the second on a smaller mesh,
so the shared static scratch keeps the first call's larger contents), on a
plain and on a batched mesh, and refused for a null mesh."""
import ctypes as C

import numpy as np
import pytest

import synth
from _util import TOL, rel, to_dev, to_host
from test_gpu_parity import make_problem, mesh_of, say

pytestmark = pytest.mark.gpu


def _noalloc(m, x, v, f, stream):
    from paper_2602_17002_amd import _lib
    L = _lib.lib()
    P = lambda t: None if t is None else C.c_void_p(t.data_ptr())
    st = L.tlfea_internal_force_noalloc(m.handle, P(x), P(v), None, P(f), C.c_void_p(stream.cuda_stream))
    return st, L.tlfea_last_error().decode()


def test_noalloc_forward_equals_forward_twice_smaller_second():
    import torch
    import oracle as O
    from paper_2602_17002_amd import BATCHED
    big = make_problem(synth.T10, "NH", True, n=(16, 12, 8), seed=90, per_elem=False)
    small = make_problem(synth.H8, "SVK", True, n=(10, 8, 6), seed=91, per_elem=False)
    multi = synth.config_multibody(8, 200, 3000, seed=92)
    s = torch.cuda.current_stream()
    for p, flags in ((big, 0), (small, 0), (multi, BATCHED), (small, 0)):
        say("noalloc", p.name, p.n_elem)
        m = mesh_of(p, flags=flags)
        assert m.info()["n_partials"] > 0
        x = to_dev(p.x)
        v = to_dev(p.v) if p.blocks[0].damped else None
        ref = m.internal_force(x, v)
        f = torch.full_like(x, float("nan"))
        st, msg = _noalloc(m, x, v, f, s)
        assert st == 0, msg
        torch.cuda.synchronize()
        assert torch.equal(f, ref)
        assert rel(to_host(f), O.internal_force(p.X, p.blocks, p.x, p.v if v is not None else None)) <= TOL


def test_noalloc_rejects_bad_arguments():
    import torch
    from paper_2602_17002_amd import _lib
    L = _lib.lib()
    assert L.tlfea_internal_force_noalloc(None, None, None, None, None, None) == -1
    p = make_problem(synth.T10, "NH", True, n=(3, 2, 2), seed=93)
    m = mesh_of(p)
    x = to_dev(p.x)
    st, msg = _noalloc(m, x, None, torch.empty_like(x), torch.cuda.current_stream())
    assert st == -1 and "v is required" in msg
    st, msg = _noalloc(m, x, to_dev(p.v), x, torch.cuda.current_stream())
    assert st == -1 and "overlaps" in msg


def test_noalloc_refuses_a_mesh_beyond_its_scratch():
    """The 256-body multibody mesh (5.5 M elements) has more shared-node
    partials than the 64 MiB scratch holds: refused before any launch."""
    import torch
    p = synth.config_c5()
    say("noalloc limit", p.name, p.n_elem)
    m = mesh_of(p, flags=0)
    assert 3 * m.info()["n_partials"] > 8 << 20
    x = to_dev(p.x)
    v = to_dev(p.v) if any(b.damped for b in p.blocks) else None
    f = torch.zeros_like(x)
    st, msg = _noalloc(m, x, v, f, torch.cuda.current_stream())
    assert st == -6 and "static scratch" in msg, msg
    torch.cuda.synchronize()
    assert not f.any()
