"""The FP64 pair kernel's own exp(-z) and 1/sqrt(x), evaluated on the device through the C
ABI (hobi_device_math), against extended-precision references over the arguments the
kernel sees: z = kappa r from 0 to 708 (denser below 50), r^2 from 1e-4 to 1e6 A^2.
Bar: 2 units in the last place of the double result."""
import numpy as np
import pytest

from paper_1301_5914_amd import hobi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return hobi.Context(0)


def _ulp_err(y, ref):
    """|y - ref| in units of the spacing of doubles at ref (ref in extended precision)."""
    r64 = ref.astype(np.float64)
    return np.abs(y.astype(np.longdouble) - ref) / np.spacing(np.abs(r64)).astype(np.longdouble)


def test_exp_neg_within_two_ulp(ctx):
    rng = np.random.default_rng(3)
    # every table entry and both ends of the reduced range: z = m ln2 / 256 and halfway
    grid = np.arange(0, 4096) * (np.log(2.0) / 512)
    z = np.concatenate([[0.0, 1e-300, 1e-12, 1e-6], grid, rng.uniform(0, 1, 100_000),
                        rng.uniform(0, 50, 200_000), rng.uniform(50, 708, 50_000), [700.0, 708.0]])
    y = hobi.hobi_device_math(ctx, hobi.HOBI_MATH_EXP_NEG, z)
    ref = np.exp(-z.astype(np.longdouble))
    err = _ulp_err(y, ref)
    print(f"exp(-z): max {float(err.max()):.2f} ulp, mean {float(err.mean()):.3f} ulp over {z.size} values", flush=True)
    assert float(err.max()) <= 2.0


def test_rsqrt_within_two_ulp(ctx):
    rng = np.random.default_rng(4)
    x = np.concatenate([10.0 ** rng.uniform(-4, 6, 300_000), [1e-4, 1.0, 2.0, 1e6],
                        np.nextafter(1.0, 2.0) * np.arange(1, 1000)])
    y = hobi.hobi_device_math(ctx, hobi.HOBI_MATH_RSQRT, x)
    ref = 1.0 / np.sqrt(x.astype(np.longdouble))
    err = _ulp_err(y, ref)
    print(f"1/sqrt(x): max {float(err.max()):.2f} ulp, mean {float(err.mean()):.3f} ulp over {x.size} values", flush=True)
    assert float(err.max()) <= 2.0


def test_domain_errors(ctx):
    for fn, bad in ((hobi.HOBI_MATH_EXP_NEG, -1.0), (hobi.HOBI_MATH_RSQRT, 0.0), (hobi.HOBI_MATH_EXP_NEG, np.nan)):
        with pytest.raises(hobi.HobiError) as ei:
            hobi.hobi_device_math(ctx, fn, np.array([1.0, bad]))
        assert ei.value.name == "HOBI_E_ARG"
