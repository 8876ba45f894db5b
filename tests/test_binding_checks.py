"""CPU tests: the Python binding checks every buffer against its descriptor
(dtype, contiguity, element count, device) before a pointer reaches the C
ABI, and raises RnError(RN_ERR_INVALID) otherwise.  Runs without a GPU:
the checks come before any call that needs a device (the plans they use are
host-only), so a handle-less stand-in context is enough."""
import numpy as np
import pytest
import torch

import paper_2201_06620_amd as rn


class FakeCtx:
    """Stand-in for rn.Context without a device handle (host-only plans)."""
    h = None
    device = 0
    _workspace = rn.Context._workspace
    _net_args = rn.Context._net_args
    _td_plan = rn.Context._td_plan

    def __init__(self):
        self._plans = {}


def td(ctx, a, b, out=None, mode="fp32_4m"):
    return rn.Context.block_tensordot(ctx, a, [2] * 4, None, b, [2] * 4, None, [3, 1], [0, 2],
                                      mode, out=out)


def status_of(excinfo):
    return excinfo.value.status


@pytest.fixture(scope="module")
def have_lib():
    try:
        rn.lib()
    except Exception as e:  # pragma: no cover - the build step makes it
        pytest.skip(f"library not built: {e}")


def test_operand_dtype_size_device(have_lib):
    ctx = FakeCtx()
    ok = torch.zeros(16, dtype=torch.complex64)
    with pytest.raises(rn.RnError) as e:          # wrong dtype for the mode
        td(ctx, ok.to(torch.complex128), ok)
    assert status_of(e) == 1 and "dtype" in str(e.value)
    with pytest.raises(rn.RnError) as e:          # too few elements for dims
        td(ctx, torch.zeros(8, dtype=torch.complex64), ok)
    assert "elements" in str(e.value)
    with pytest.raises(rn.RnError) as e:          # not contiguous
        td(ctx, torch.zeros(32, dtype=torch.complex64)[::2], ok)
    assert "contiguous" in str(e.value)
    with pytest.raises(rn.RnError) as e:          # host tensor of the right shape
        td(ctx, ok, ok)
    assert "GPU" in str(e.value)
    with pytest.raises(rn.RnError) as e:          # complex64 operands with FP64 mode
        td(ctx, ok, ok, mode="fp64")
    assert "dtype" in str(e.value)


def test_network_tensor_and_result_checks(have_lib):
    ctx = FakeCtx()
    t2 = torch.zeros(4, dtype=torch.complex64)
    with pytest.raises(rn.RnError) as e:          # 3 elements for a rank-2 tensor
        rn.Context._net_args(ctx, [torch.zeros(3, dtype=torch.complex64), t2],
                             [[1, 2], [1, 2]], "fp32_4m")
    assert status_of(e) == 1 and "elements" in str(e.value)
    with pytest.raises(rn.RnError) as e:          # complex128 tensors with an FP32 mode
        rn.Context._net_args(ctx, [t2.to(torch.complex128), t2], [[1, 2], [1, 2]], "fp32_4m")
    assert "dtype" in str(e.value)
    with pytest.raises(rn.RnError):               # label lists and tensors differ in number
        rn.Context._net_args(ctx, [t2], [[1, 2], [1, 2]], "fp32_4m")
    with pytest.raises(rn.RnError) as e:          # amp too short
        rn._check_amp_slices(torch.zeros(1, dtype=torch.float64), None, 0, 0)
    assert "elements" in str(e.value)
    with pytest.raises(rn.RnError) as e:          # slices shorter than 2 * 2^nsliced
        rn._check_amp_slices(torch.zeros(2, dtype=torch.float64),
                             torch.zeros(15, dtype=torch.float64), 3, 0)
    assert "16" in str(e.value)
    with pytest.raises(rn.RnError) as e:          # amp of the wrong dtype
        rn._check_amp_slices(torch.zeros(2, dtype=torch.float32), None, 0, 0)
    assert "dtype" in str(e.value)


def test_workspace_check(have_lib):
    ctx = FakeCtx()
    with pytest.raises(rn.RnError) as e:
        rn.Context._workspace(ctx, 64, torch.zeros(64, dtype=torch.uint8))
    assert "GPU" in str(e.value)
    with pytest.raises(rn.RnError):
        rn.Context._workspace(ctx, 64, torch.zeros(128, dtype=torch.uint8)[::2])


def test_server_submit_checks_host_sizes(have_lib):
    srv = rn.Server.__new__(rn.Server)
    srv.s = None
    with pytest.raises(rn.RnError) as e:
        rn.Server.submit(srv, [np.zeros(3, dtype=np.complex64)], [[1, 2]], [], (), "fp32_4m")
    assert "elements" in str(e.value)
    srv.s = None


def test_axes_lengths_must_agree(have_lib):
    """The library reads len(axes_a) entries of both axis arrays: a shorter
    axes_b is refused in the binding, before any library call."""
    with pytest.raises(rn.RnError) as e:
        rn.plan_block_tensordot([2] * 4, None, [2] * 4, None, [3, 1], [0], "fp32_4m")
    assert status_of(e) == 1 and "paired" in str(e.value)
    ok = torch.zeros(16, dtype=torch.complex64)
    with pytest.raises(rn.RnError) as e:
        rn.Context.block_tensordot(FakeCtx(), ok, [2] * 4, None, ok, [2] * 4, None, [3, 1],
                                   [0, 2, 1], "fp32_4m")
    assert "paired" in str(e.value)
    with pytest.raises(rn.RnError) as e:          # one problem of a batch
        rn.plan_batch_workspace(None, [(None, [2] * 4, None, None, [2] * 4, None, [3, 1], [0, 2]),
                                       (None, [2] * 4, None, None, [2] * 4, None, [3], [0, 2])])
    assert "paired" in str(e.value)
    with pytest.raises(rn.RnError) as e:
        rn.block_footprint([2] * 4, None, [2] * 4, None, [3, 1, 2], [0, 2])
    assert "paired" in str(e.value)


def test_plan_cache_matches_uncached_plan(have_lib):
    """Repeated block tensordots on one shape reuse the handle's cached plan;
    the cached C shape and workspace equal a fresh plan's, distinct shapes and
    modes get distinct entries, and the buffer checks still run on every call."""
    ctx = FakeCtx()
    shapes = [([2] * 4, None, [2] * 4, None, [3, 1], [0, 2], "fp32_4m"),
              ([2] * 4, None, [2] * 4, None, [3, 1], [0, 2], "fp64"),
              ([2] * 6, [2, 1, 1, 1, 1, 1], [2] * 5, [1, 2, 1, 1, 1], [5, 0], [1, 3], "bf16x3")]
    for sh in shapes:
        e1 = ctx._td_plan(*sh)
        assert ctx._td_plan(*sh) is e1
        cd, cg, ws, fl = rn.plan_block_tensordot(*sh)
        assert (e1["cdims"], e1["cgrid"], e1["ws"], e1["flops"]) == (cd, cg, ws, fl)
        assert e1["n"] == int(np.prod(cd))
    assert len(ctx._plans) == len(shapes)
    ok = torch.zeros(16, dtype=torch.complex64)
    for _ in range(2):                            # cached shape, wrong operand size
        with pytest.raises(rn.RnError) as e:
            td(ctx, torch.zeros(8, dtype=torch.complex64), ok)
        assert "elements" in str(e.value)
