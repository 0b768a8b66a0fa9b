"""The tile-shape autotuner's host logic (no GPU): the crossover choice, the p(n)
table it hands to Eq. 10, and the check that a stored policy fits the GPU."""
import json

from paper_2205_12182_amd import autotune as A


def rec(npad, ms128, ms256, n=None, k=512):
    return {"npad_mean": npad, "n_mean": npad - 30 if n is None else n, "submatrices": k,
            "tile128": {"ms_per_launch": ms128}, "tile256x128": {"ms_per_launch": ms256}}


def test_choose_crossover():
    # the large tiles are faster from 460 up: the policy starts there (rounded down to 64)
    recs = [rec(378, 0.14, 0.17), rec(460, 0.20, 0.19), rec(535, 0.26, 0.25), rec(900, 0.9, 0.8)]
    assert A.choose(recs) == 448
    # a win below a loss does not count: only the wins above the last loss
    recs = [rec(378, 0.14, 0.13), rec(460, 0.19, 0.20), rec(535, 0.26, 0.25), rec(900, 0.9, 0.8)]
    assert A.choose(recs) == 512
    # never faster: the "never" threshold
    assert A.choose([rec(378, 0.14, 0.17), rec(900, 0.8, 0.9)]) == A.NEVER
    # order of the records does not matter
    recs = [rec(900, 0.9, 0.8), rec(378, 0.14, 0.17), rec(535, 0.26, 0.25), rec(460, 0.20, 0.19)]
    assert A.choose(recs) == 448


def test_rate_table_follows_policy_and_paper_accounting():
    """p(n) = 2 n^3 per product and submatrix over the launch time of the tile
    shape the policy uses at that size, ascending in n."""
    recs = [rec(900, 2.0, 1.0, n=870, k=256), rec(378, 0.2, 0.25, n=341, k=512)]
    pol = {"big_tile_min_npad": 448, "measurements": recs}
    table = A.rate_table(pol)
    assert [n for n, _ in table] == [341.0, 870.0]
    # n = 341 uses 128 x 128 tiles (0.2 ms), n = 870 the large tiles (1.0 ms)
    assert abs(table[0][1] - 2 * 512 * 341.0 ** 3 / 0.2e-3 / 1e12) < 1e-9
    assert abs(table[1][1] - 2 * 256 * 870.0 ** 3 / 1.0e-3 / 1e12) < 1e-9


def test_policy_applies_to_its_architecture_only():
    digest = A.gemm_sources_digest()
    pol = {"big_tile_min_npad": 448,
           "target": {"gfx_arch": "gfx950", "hip_version": "7.0", "kernel_sha256": digest}}
    assert A.policy_applies(pol, "gfx950") == (True, "")
    ok, note = A.policy_applies(pol, "gfx942")
    assert not ok and "gfx942" in note
    pol["target"]["kernel_sha256"] = "0" * 16
    ok, note = A.policy_applies(pol, "gfx950")
    assert ok and "changed" in note
    assert A.policy_applies({"big_tile_min_npad": 448}, "gfx950") == (True, "")


def test_committed_policy_is_well_formed():
    with open(A.POLICY_PATH) as fh:
        pol = json.load(fh)
    assert pol["big_tile_min_npad"] % 64 == 0 or pol["big_tile_min_npad"] == A.NEVER
    assert A.choose(pol["measurements"]) == pol["big_tile_min_npad"]
    table = A.rate_table(pol)
    assert len(table) == len(A.RADII) and all(r > 0 for _, r in table)
