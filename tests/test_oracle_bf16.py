"""Pin the oracle's BF16 rounding against torch's own float32 -> bfloat16
conversion (a separate implementation) and against hand-worked bit patterns."""
import numpy as np
import torch

from oracle.bf16 import round_bf16


def test_round_bf16_matches_torch_on_random_and_edge_values():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(100000).astype(np.float32),
        (rng.standard_normal(10000) * 1e30).astype(np.float32),
        (rng.standard_normal(10000) * 1e-30).astype(np.float32),
        np.array([0.0, -0.0, 1.0, -1.0, 3.4e38, -3.4e38, 1e-45, np.inf, -np.inf], np.float32),
    ])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = round_bf16(x)
    np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))


def test_round_bf16_ties_go_to_even():
    # 1 + 2^-8 lies halfway between BF16 neighbours 1 and 1 + 2^-7: rounds to 1 (even)
    # 1 + 3*2^-8 lies halfway between 1 + 2^-7 and 1 + 2^-6: rounds up to the even one
    x = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20], np.float32)
    got = round_bf16(x)
    np.testing.assert_array_equal(got, np.array([1.0, 1 + 2 ** -6, 1 + 2 ** -7], np.float32))


def test_round_bf16_nan_stays_nan():
    assert np.isnan(round_bf16(np.array([np.nan], np.float32)))[0]
