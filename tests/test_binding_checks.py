"""The binding's argument checks (CPU only, no library call is reached): every array handed to the
C ABI must be a contiguous GPU tensor of the dtype and element count the header states, on the
context's device; anything else raises ValueError before the call."""
import pytest
import torch

from paper_2306_17537_amd import ie

CTX = 0x5EED  # a fake handle: the checks reject the arrays before the library sees it
NN = 0x5EEE


@pytest.fixture(autouse=True)
def fake_handles():
    ie._CTX[CTX] = ((4, 3, 2), 0)
    ie._NN[NN] = (14, 6)
    yield
    ie._CTX.pop(CTX, None)
    ie._NN.pop(NN, None)


N = 4 * 3 * 2


def _field(dtype=torch.complex128, n=3 * N):
    return torch.zeros(n, dtype=dtype)


def test_matvec_rejects_wrong_dtype_size_layout_and_host_memory():
    s6 = torch.zeros(6 * N, dtype=torch.float64)
    with pytest.raises(ValueError, match="dtype"):
        ie.ie_matvec(CTX, s6, _field(torch.complex64), _field(), precision=ie.IE_FP64)
    with pytest.raises(ValueError, match="dtype"):
        ie.ie_matvec(CTX, s6, _field(), _field(), precision=ie.IE_MIXED)
    with pytest.raises(ValueError, match="elements"):
        ie.ie_matvec(CTX, s6, _field(n=3 * N - 1), _field())
    with pytest.raises(ValueError, match="sigma6.*elements"):
        ie.ie_matvec(CTX, torch.zeros(6 * N + 6, dtype=torch.float64), _field(), _field())
    with pytest.raises(ValueError, match="sigma6.*dtype"):
        ie.ie_matvec(CTX, s6.float(), _field(), _field())
    strided = torch.zeros(2 * 3 * N, dtype=torch.complex128)[::2]
    with pytest.raises(ValueError, match="contiguous"):
        ie.ie_matvec(CTX, s6, strided, _field())
    with pytest.raises(ValueError, match="GPU"):
        ie.ie_matvec(CTX, s6, _field(), _field())
    with pytest.raises(ValueError, match="GPU"):
        ie.ie_matvec_noalloc(CTX, s6, _field(), _field())
    with pytest.raises(ValueError, match="required"):
        ie.ie_matvec(CTX, None, _field(), _field(), form=ie.IE_CIE)
    with pytest.raises(ValueError, match="torch tensor"):
        ie.ie_matvec(CTX, s6, [0.0] * 3 * N, _field())


def test_solvers_and_receivers_check_their_arrays():
    s6 = torch.zeros(6 * N, dtype=torch.float64)
    with pytest.raises(ValueError, match="b: dtype"):
        ie.ie_gmres(CTX, s6, _field(torch.complex64), _field())
    with pytest.raises(ValueError, match="x: .*elements"):
        ie.ie_gmres(CTX, s6, _field(), _field(n=N))
    with pytest.raises(ValueError, match="E0"):
        ie.ie_background_field(CTX, [((0, 0, 5.0), (0, 0, 1), "magnetic")], _field(n=1))
    with pytest.raises(ValueError, match="E: dtype"):
        ie.ie_receivers(CTX, s6, [], _field(torch.complex64), [[0, 0, 9.0]])
    g = ie.make_grid((4, 3, 2), 0.25, (0, 0, 0))
    prob = dict(grid=g, sigma6=s6, sources=[((0, 0, 5.0), (0, 0, 1), "magnetic")],
                E_total=_field(), E_anom=_field(n=5))
    with pytest.raises(ValueError, match="problem 0 E_anom"):
        ie.ie_dd_solve([CTX], [prob], ie.dd_opts())
    prob["E_anom"] = None
    prob["E_total"] = _field(n=3 * N + 3)
    with pytest.raises(ValueError, match="problem 0 E_total"):
        ie.ie_dd_solve([CTX], [prob], ie.dd_opts())


def test_network_calls_check_their_arrays():
    x = torch.zeros((1, 2, 3, 4, 14), dtype=torch.bfloat16)
    y = torch.zeros((1, 2, 3, 4, 6), dtype=torch.float32)
    with pytest.raises(ValueError, match="x: dtype"):
        ie.ie_nn_forward(NN, x.float(), y)
    with pytest.raises(ValueError, match="y: .*elements"):
        ie.ie_nn_forward(NN, x, torch.zeros((1, 2, 3, 4, 5), dtype=torch.float32))
    with pytest.raises(ValueError, match="target: dtype"):
        ie.ie_nn_train_step(NN, x, y.double(), 1e-3)
    with pytest.raises(ValueError, match="x: expected"):
        ie.ie_nn_forward(NN, x[0], y)
    with pytest.raises(ValueError, match="GPU"):
        ie.ie_nn_forward(NN, x, y)
    with pytest.raises(ValueError, match="x: .*elements"):
        ie.ie_nn_features(CTX, torch.zeros(6 * N, dtype=torch.float64), _field(),
                          torch.zeros((N, 13), dtype=torch.bfloat16))
    with pytest.raises(ValueError, match="C: dtype"):
        ie.ie_nn_gemm(torch.zeros(6, dtype=torch.bfloat16), torch.zeros(6, dtype=torch.bfloat16),
                      torch.zeros(4, dtype=torch.float64), 2, 2, 3)


def test_every_wrapper_marshals_valid_arrays_through_to_the_library(monkeypatch):
    """With the device check and the library replaced by stand-ins, each wrapper turns valid
    arrays into one library call with the C name (catches marshalling mistakes on the CPU)."""
    import ctypes as C
    calls = []

    class FakeLib:
        def __getattr__(self, name):
            def f(*args):
                calls.append(name)
                return 0
            return f

    monkeypatch.setattr(ie, "lib", lambda: FakeLib())
    monkeypatch.setattr(ie, "_ptrs", lambda device, *a: [None if x is None else
                                                          C.c_void_p(x[1].data_ptr()) for x in a])
    monkeypatch.setattr(ie, "_stream", lambda stream: C.c_void_p(0))
    s6 = torch.zeros(6 * N, dtype=torch.float64)
    src = [((0, 0, 5.0), (0, 0, 1), "magnetic")]
    ie.ie_background_field(CTX, src, _field())
    ie.ie_matvec(CTX, s6, _field(), _field())
    ie.ie_matvec_noalloc(CTX, s6, _field(torch.complex64), _field(torch.complex64),
                         precision=ie.IE_MIXED)
    ie.ie_gmres(CTX, s6, _field(), _field())
    g = ie.make_grid((4, 3, 2), 0.25, (0, 0, 0))
    ie.ie_dd_solve([CTX], [dict(grid=g, sigma6=s6, sources=src, E_total=_field())], ie.dd_opts())
    ie.ie_receivers(CTX, s6, src, _field(), [[0, 0, 9.0]])
    x = torch.zeros((1, 2, 3, 4, 14), dtype=torch.bfloat16)
    y = torch.zeros((1, 2, 3, 4, 6), dtype=torch.float32)
    ie.ie_nn_forward(NN, x, y)
    ie.ie_nn_backward(NN, x, y.clone(), y)
    ie.ie_nn_train_step(NN, x, y, 1e-3)
    ie.ie_nn_gemm(torch.zeros(6, dtype=torch.bfloat16), torch.zeros(6, dtype=torch.bfloat16),
                  torch.zeros(4, dtype=torch.float32), 2, 2, 3)
    ie.ie_nn_features(CTX, s6, _field(), torch.zeros((N, 14), dtype=torch.bfloat16))
    ie.ie_nn_target(CTX, _field(), _field(), torch.zeros((N, 6), dtype=torch.float32))
    ie.ie_nn_predict(CTX, NN, s6, _field(), _field())
    ie.ie_nn_guess(CTX, NN, s6, _field(), _field())
    assert calls == ["ie_background_field", "ie_matvec", "ie_matvec_noalloc", "ie_gmres",
                     "ie_dd_solve", "ie_receivers", "ie_nn_forward", "ie_nn_backward",
                     "ie_nn_train_step", "ie_nn_gemm", "ie_nn_features", "ie_nn_target",
                     "ie_nn_predict", "ie_nn_guess"]
