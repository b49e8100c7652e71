"""Host-side logic of bench.py (no GPU): the split of a batch over properties and
the per-launch shares of the per-iteration state floor."""
import pytest

import bench
import ldgen


def test_split_shares_keep_every_property():
    props = ldgen.CONFIGS["deep"]["props"]
    for B in (6, 7, 50, 506, 4044, 5000):
        sh = bench.split_shares(B, props)
        assert sum(sh) == B and min(sh) >= 1
    assert bench.split_shares(4044, props) == props
    with pytest.raises(ValueError):
        bench.split_shares(4, props)


@pytest.mark.parametrize("name", ["wide", "base", "deep", "tiny_conv2"])
def test_floor_shares_add_up_to_the_state_floor(name):
    inst = ldgen.make_instance(name, **({"props": [1] * len(ldgen.CONFIGS[name]["props"])}
                                        if len(ldgen.CONFIGS[name]["props"]) > 1 else {"B": 1}))
    n = len(inst.layers)
    kinds = [100 + k for k in range(1, n)] + [300 + k for k in range(1, n)]
    B = 7
    assert sum(bench.floor_share(inst, k, B) for k in kinds) == bench.state_floor(inst, B)
