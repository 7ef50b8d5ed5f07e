"""Host-side checks of the Python binding (no GPU): the tensor validation that
runs before any pointer reaches the library."""
import pytest

from paper_1910_07054_amd import hfd

torch = pytest.importorskip("torch")


def _check(t, **kw):
    args = dict(name="m", nz=2, ny=3, nx=4, fp64=False, batch_max=4, n_geom=1)
    args.update(kw)
    return hfd.check_field_tensor(t, **args)


def test_validator_rejects_host_tensors_and_non_tensors():
    with pytest.raises(ValueError, match="GPU"):
        _check(torch.zeros((1, 3, 2, 3, 4)))
    with pytest.raises(TypeError):
        _check([[0.0]])


class _FakeCuda:
    """A stand-in with the attributes the validator reads, so that the rules
    after the device check run on a machine without a GPU."""

    def __init__(self, t, device="cuda:0"):
        self._t = t
        self.is_cuda = True
        self.device = torch.device(device)

    def __getattr__(self, k):
        return getattr(self._t, k)


@pytest.fixture()
def fake(monkeypatch):
    # make isinstance(x, torch.Tensor) accept the stand-in
    real = torch.Tensor

    class Meta(type):
        def __instancecheck__(cls, obj):
            return isinstance(obj, (_FakeCuda, real))
    monkeypatch.setattr(torch, "Tensor", Meta("Tensor", (), {}))
    return _FakeCuda


def test_validator_rules(fake):
    ok = fake(torch.zeros((2, 3, 2, 3, 4)))
    assert _check(ok) == 2
    assert _check(ok, n_geom=2) == 2
    with pytest.raises(ValueError, match="float64"):
        _check(ok, fp64=True)
    with pytest.raises(ValueError, match="float32"):
        _check(fake(torch.zeros((2, 3, 2, 3, 4), dtype=torch.float64)))
    with pytest.raises(ValueError, match="shape"):
        _check(fake(torch.zeros((2, 3, 2, 4, 3))))
    with pytest.raises(ValueError, match="shape"):
        _check(fake(torch.zeros((3, 2, 3, 4))))
    with pytest.raises(ValueError, match="contiguous"):
        _check(fake(torch.zeros((2, 3, 2, 4, 3)).transpose(3, 4)))
    with pytest.raises(ValueError, match="contiguous"):
        _check(fake(torch.zeros((1, 3, 2, 3, 4)).expand(2, 3, 2, 3, 4)))
    with pytest.raises(ValueError, match="batch"):
        _check(fake(torch.zeros((5, 3, 2, 3, 4))))
    with pytest.raises(ValueError, match="multiple"):
        _check(fake(torch.zeros((3, 3, 2, 3, 4))), n_geom=2)
    with pytest.raises(ValueError, match="differs"):
        _check(ok, batch=1)
    with pytest.raises(ValueError, match="plan on"):
        _check(ok, device=torch.device("cuda:1"))
