"""The Python binding refuses sizes that the C ABI's int32 arguments cannot
hold, before any library call (ctypes would truncate them silently: a
tensor of 2^32 + 5 elements would be processed as 5). No GPU and no large
allocation: the tensors are stand-ins whose numel() reports the size."""
import pytest

import paper_2103_15217_amd.et as et

BIG = (1 << 32) + 5


class FakeTensor:
    def __init__(self, numel):
        self._n = numel
        self.device = "cuda:0"

    def numel(self):
        return self._n

    def data_ptr(self):  # never reached: the size check comes first
        raise AssertionError("library called with an oversized argument")


class FakeCtx:
    handle = None
    device = 0


@pytest.fixture(autouse=True)
def no_device_checks(monkeypatch):
    monkeypatch.setattr(et, "_dev", lambda t, dtype, name: t)

    def no_lib(*a, **k):
        raise AssertionError("library called with an oversized argument")

    monkeypatch.setattr(et, "_lib", type("L", (), {"__getattr__": lambda self, name: no_lib})())


def test_i32_helper():
    assert et._i32(5, "x") == 5
    assert et._i32(et.INT32_MAX, "x") == et.INT32_MAX
    for bad in (-1, et.INT32_MAX + 1, BIG):
        with pytest.raises(ValueError):
            et._i32(bad, "x")
    with pytest.raises(ValueError):
        et._i32(et.NODE_MAX + 1, "x", et.NODE_MAX)


@pytest.mark.parametrize("size", [BIG, et.LIST_MAX + 1])
def test_list_rank_length(size):
    with pytest.raises(ValueError, match="list length"):
        et.et_list_rank(FakeTensor(size), FakeTensor(1), ctx=FakeCtx())
    with pytest.raises(ValueError, match="list length"):
        et.et_list_scan(FakeTensor(size), FakeTensor(size), FakeTensor(1), ctx=FakeCtx())


def test_list_heads():
    with pytest.raises(ValueError, match="heads"):
        et.et_list_rank(FakeTensor(10), FakeTensor(BIG), ctx=FakeCtx())


@pytest.mark.parametrize("size", [BIG, et.NODE_MAX + 1])
def test_tree_sizes(size):
    with pytest.raises(ValueError, match="tree size"):
        et.et_tree_build(FakeTensor(size), ctx=FakeCtx())
    with pytest.raises(ValueError, match="tree size"):
        et.et_levels(FakeTensor(size), ctx=FakeCtx())
    with pytest.raises(ValueError, match="tree size"):
        et.et_lca_naive(FakeTensor(size), FakeTensor(size), FakeTensor(4), FakeTensor(4), ctx=FakeCtx())
    with pytest.raises(ValueError, match="tree size"):
        et.et_tree_build_edges(FakeTensor(size - 1), FakeTensor(size - 1), size, 0, ctx=FakeCtx())


def test_batch_sizes():
    with pytest.raises(ValueError, match="batch size"):
        et.et_tree_build_batch(FakeTensor(et.NODE_MAX), FakeTensor(3), ctx=FakeCtx())
    with pytest.raises(ValueError, match="number of trees"):
        et.et_tree_build_batch(FakeTensor(10), FakeTensor(BIG), ctx=FakeCtx())


def test_bridge_sizes():
    with pytest.raises(ValueError, match="vertex count"):
        et.et_bridges(FakeTensor(BIG), FakeTensor(4), ctx=FakeCtx())
    with pytest.raises(ValueError, match="CSR slot count"):
        et.et_bridges(FakeTensor(11), FakeTensor(BIG), ctx=FakeCtx())
    with pytest.raises(ValueError, match="CSR slot count"):
        et.et_bridges_ck(FakeTensor(11), FakeTensor(BIG), ctx=FakeCtx())
    with pytest.raises(ValueError, match="total CSR slot count"):
        et.et_bridges_batch(row_ptr=FakeTensor(12), col=FakeTensor(BIG), voff=FakeTensor(3), soff=FakeTensor(3),
                            slots=[BIG - 1, 1], ctx=FakeCtx())
