"""The stored full-size references (tests/golden/fullsize_refs.npz) are current: each entry's
input hash matches the workload the recipes generate now, so the full-size GPU tests use them
instead of recomputing."""

import pytest

import synth
from golden_refs import M, current


@pytest.mark.parametrize("name", M.WORKLOADS)
def test_stored_references_are_current(name):
    w = synth.workload(name)
    Y = M.targets(w)
    assert current(name, w, Y), f"{name}: rerun python tests/golden/make_fullsize_refs.py"
    if name == "grad":
        assert current("grad", w, Y, "ghash", M.grad_points(w.D).tobytes())
