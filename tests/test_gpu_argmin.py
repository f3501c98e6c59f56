"""ivde_argmin on hand-made cost tables: the lowest label among the minima
of each row, NaN never winning, an all-NaN (or all-infinite) row giving
label 0.  Integer work, so compared exactly with numpy's first-occurrence
argmin of the same values (NaN replaced by +inf), in FP32 and FP16, for
level counts that fill the vector loads and ones that do not, row counts
that leave a ragged last block, and a base address that is not 16-byte
aligned (the scalar path)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1909_02294_amd import ivde  # noqa: E402


def _expected(c):
    x = c.astype(np.float64)
    x[np.isnan(x)] = np.inf
    return np.argmin(x, axis=1).astype(np.int32)


def _table(rows, L, dtype, seed):
    rng = np.random.default_rng(seed)
    # few distinct values, so most rows hold ties for the minimum
    c = rng.integers(0, 6, (rows, L)).astype(np.float32) / 8.0
    if rows > 3:
        c[1, :] = np.nan
        c[2, :] = np.inf
        c[3, ::2] = np.nan
    return c.astype(dtype)


@pytest.mark.parametrize("half", [False, True])
@pytest.mark.parametrize("L", [1, 3, 4, 63, 64, 65, 256, 300])
@pytest.mark.parametrize("rows", [1, 5, 17, 1000])
def test_argmin_exact(rows, L, half):
    print(f"[case] argmin rows={rows} L={L} half={half}", flush=True)
    dt = np.float16 if half else np.float32
    c = _table(rows, L, dt, seed=rows * 1000 + L)
    got = ivde.argmin(torch.from_numpy(c).cuda()).cpu().numpy()
    np.testing.assert_array_equal(got, _expected(c))


@pytest.mark.parametrize("half", [False, True])
def test_argmin_unaligned_base(half):
    """A table starting one element into its allocation: 4-byte (FP32) or
    2-byte (FP16) aligned only, so the kernel reads element by element."""
    print(f"[case] argmin unaligned half={half}", flush=True)
    dt = np.float16 if half else np.float32
    rows, L = 37, 256
    flat = _table(1, rows * L + 1, dt, seed=5).ravel()
    dev = torch.from_numpy(flat).cuda()
    view = dev[1:].view(rows, L)
    assert view.data_ptr() % 16 != 0
    got = ivde.argmin(view).cpu().numpy()
    np.testing.assert_array_equal(got, _expected(flat[1:].reshape(rows, L)))


def test_argmin_rejects_misread_tables():
    print("[case] argmin argument checks", flush=True)
    c = torch.zeros((6, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        ivde.argmin(c.double())
    with pytest.raises(ValueError):
        ivde.argmin(c.t())
    with pytest.raises(ValueError):
        ivde.argmin(c, out=torch.empty(6, dtype=torch.int64, device="cuda"))
    with pytest.raises(ValueError):
        ivde.argmin(c, out=torch.empty(5, dtype=torch.int32, device="cuda"))
