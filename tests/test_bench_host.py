"""Host-side bookkeeping of bench.py (no GPU): the counter-traffic lookup is
keyed to the operator's sources, the p-multigrid byte model adds up and uses
the split-form residual on the order >= 5 levels only, and the dealiased
advection's matrix-core count follows its tile structure."""

import os

import pytest

import bench


def _fake_tree(tmp_path):
    csrc = tmp_path / "paper_2501_13240_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in bench.OPERATOR_SOURCES:
        (csrc / name).write_text(f"// {name}\n")
    (tmp_path / "profiles").mkdir()
    return csrc


def test_counter_traffic_follows_the_operator_sources(tmp_path, monkeypatch):
    csrc = _fake_tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    sha = bench.operator_sources_sha256()
    prof = tmp_path / "profiles" / "ax_N7_convection_box_traffic.txt"
    prof.write_text("# header\n| table | row |\noperator sources sha256: " + sha +
                    "\ntraffic_bytes_per_launch: 123456\n")
    assert bench.counter_traffic() == 123456.0
    # any operator source changed since the counters were taken: no figure
    (csrc / bench.OPERATOR_SOURCES[1]).write_text("// changed\n")
    assert bench.counter_traffic() is None
    # no profile at all
    prof.unlink()
    assert bench.counter_traffic() is None


def test_committed_profile_names_the_hash_key():
    """The committed counter summary carries the key counter_traffic reads."""
    path = os.path.join(bench.ROOT, "profiles", "ax_N7_convection_box_traffic.txt")
    keys = [line.split(":", 1)[0].strip() for line in open(path) if ":" in line
            and not line.startswith(("|", "#", " "))]
    assert "operator sources sha256" in keys and "traffic_bytes_per_launch" in keys


def test_pmg_byte_model_adds_up():
    total, parts = bench.pmg_cube_iteration_bytes()
    assert total == pytest.approx(sum(parts.values()))
    split = [k for k in parts if k.startswith("residual, split form")]
    gather = [k for k in parts if k.startswith("residual sums")]
    assert len(split) == 1 and len(gather) == 1
    # level 0 (N = 9) alone takes the split form; its share with 2 (m - 1) + 2
    # residuals of 8 n_1 + 8 (n_L - n_1) + 8 (n_f - n_1) + 4 n_f bytes
    E, N, nel = 32 ** 3, 9, 32
    nL, nf = E * (N + 1) ** 3, (nel * N + 1) ** 3
    n1 = E * (N - 1) ** 3 + 6 * nel * nel * (N - 1) ** 2
    m = 4
    want = (2 * (m - 1) + 2) * (8 * n1 + 8 * (nL - n1) + 8 * (nf - n1) + 4 * nf)
    assert parts[split[0]] == pytest.approx(want)
    # a cycle without an order >= 5 level has no split-form residual
    _, parts_low = bench.pmg_cube_iteration_bytes(nel=4, orders=(4, 2, 1))
    assert not any(k.startswith("residual, split form") for k in parts_low)


@pytest.mark.parametrize("N", [5, 7, 9])
def test_dealias_mfma_count_grows_with_fields(N):
    one = bench.dealias_mfma_per_element(N, 1)
    four = bench.dealias_mfma_per_element(N, 4)
    assert 0 < one < four < 4 * one
