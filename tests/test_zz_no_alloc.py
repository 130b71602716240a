"""dpf_build_ybus_noalloc (temporaries in the library's static per-device array)
against dpf_build_ybus (hipMalloc'd temporaries): identical CSR pattern, values
and row bound, on two calls in a row with the second grid smaller than the
first, so that a stale first-call array would show; and the size bound."""

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_28203_amd as m
    m.lib()
    return m


def _same(a, b):
    assert a.nnz == b.nnz and a.max_row_nnz == b.max_row_nnz
    assert torch.equal(a.row_ptr, b.row_ptr)
    assert torch.equal(a.col_idx, b.col_idx)
    assert torch.equal(a.val, b.val)  # same kernels, same summation order: bit for bit


def test_noalloc_build_equals_the_allocating_build_twice(dpf):
    big = synth.config2(B=1)["grid"]      # 9241 buses, 16049 branches
    small = synth.config0(3)["grid"]      # 14 buses
    for g in (big, small):
        print(f"no-alloc Y-bus build, n={g.n_bus}, branches={len(g.f)}", flush=True)
        ref = dpf.build_ybus(g.n_bus, g.f, g.t, g.r, g.x, g.b)
        got = dpf.build_ybus(g.n_bus, g.f, g.t, g.r, g.x, g.b, noalloc=True)
        torch.cuda.synchronize()
        _same(got, ref)
    # parallel branches summed (a duplicate of branch 3 on the small grid), after the larger call
    f = np.append(small.f, small.f[3]); t = np.append(small.t, small.t[3])
    r = np.append(small.r, 0.05); x = np.append(small.x, 0.2); b = np.append(small.b, 0.01)
    _same(dpf.build_ybus(small.n_bus, f, t, r, x, b, noalloc=True), dpf.build_ybus(small.n_bus, f, t, r, x, b))


def test_noalloc_build_checks_its_bound_and_inputs(dpf):
    # 400 000 buses in a chain: about 22.4 MB of temporaries > 16 MiB, rejected before device work
    n = 400000
    f = np.arange(n - 1, dtype=np.int32); t = f + 1
    ones = np.full(n - 1, 0.1)
    with pytest.raises(dpf.DPFError) as e:
        dpf.build_ybus(n, f, t, ones, ones, ones * 0, noalloc=True)
    assert e.value.code == dpf.binding.DPF_EINVAL and "static scratch" in str(e.value)
    # bad branches are reported as by dpf_build_ybus, and the next call is unaffected
    with pytest.raises(dpf.DPFError) as e:
        dpf.build_ybus(3, [0], [5], [0.1], [0.1], [0.0], noalloc=True)
    assert e.value.code == dpf.binding.DPF_EINVAL
    g = synth.config0(1)["grid"]
    _same(dpf.build_ybus(g.n_bus, g.f, g.t, g.r, g.x, g.b, noalloc=True),
          dpf.build_ybus(g.n_bus, g.f, g.t, g.r, g.x, g.b))
