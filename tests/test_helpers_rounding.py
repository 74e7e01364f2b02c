"""The test-side rounding helper agrees with numpy's and torch's own casts."""
import numpy as np
import torch

from tests.helpers import round_to


def test_round_to_matches_library_casts():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        [0.0, -0.0, 1.0, 65504.0, 6.1e-5, 1e-8]])
    np.testing.assert_array_equal(round_to(x, "f16"), x.astype(np.float16).astype(np.float64))
    np.testing.assert_array_equal(round_to(x, "f32"), x.astype(np.float32).astype(np.float64))
    # float32 inputs: bfloat16 rounding equals torch's float32 -> bfloat16 cast
    f = x.astype(np.float32).astype(np.float64)
    t = torch.from_numpy(f.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_to(f, "bf16"), t)


def test_bf16_from_double_is_single_rounding():
    # halfway between two bf16 values after a first rounding to float32 would
    # mislead a naive double rounding; round-to-odd keeps it correct
    one = 1.0
    ulp = 2.0**-7
    x = np.array([one + ulp / 2 + 2.0**-40, one + ulp / 2 - 2.0**-40, one + ulp / 2])
    np.testing.assert_array_equal(round_to(x, "bf16"), [one + ulp, one, one])
