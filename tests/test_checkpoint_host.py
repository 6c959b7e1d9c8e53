"""Host-side parts of checkpoint / resume (no GPU): the GKTL record of a resumed run and
the checkpoint format's version check."""
import pytest
import torch

from paper_2005_09323_amd.ensemble import CHECKPOINT_VERSION, Ensemble
from paper_2005_09323_amd.rare import GktlRun


def _run(col0, periods, n=4, k=0.5, tau=8, base=0):
    anc = torch.arange(base, base + periods * n, dtype=torch.int32).reshape(periods, n) % n
    ints = torch.arange(periods * n, dtype=torch.float64).reshape(periods, n) + base
    lnr = torch.arange(periods, dtype=torch.float64) + base
    return GktlRun(k, tau, periods, col0, anc, ints, lnr)


def test_then_joins_a_continuation():
    first = _run(1, 3)
    second = _run(1 + 3 * 8, 2, base=100)
    whole = first.then(second)
    assert whole.n_periods == 5 and whole.col0 == 1 and whole.t_a == 40
    assert torch.equal(whole.ancestors[:3], first.ancestors) and torch.equal(whole.ancestors[3:], second.ancestors)
    assert torch.equal(whole.integrals[3:], second.integrals)
    assert torch.equal(whole.ln_r, torch.cat([first.ln_r, second.ln_r]))  # what its SCGF sums over T_a = 40


@pytest.mark.parametrize("bad", ["gap", "k", "tau"])
def test_then_rejects_what_is_not_a_continuation(bad):
    first = _run(1, 3)
    if bad == "gap":
        second = _run(1 + 3 * 8 + 1, 2)
    elif bad == "k":
        second = GktlRun(0.25, 8, 2, 25, first.ancestors[:2], first.integrals[:2], first.ln_r[:2])
    else:
        second = GktlRun(0.5, 16, 2, 25, first.ancestors[:2], first.integrals[:2], first.ln_r[:2])
    with pytest.raises(ValueError):
        first.then(second)


def test_restore_checks_the_format_version_first():
    with pytest.raises(ValueError, match="version"):
        Ensemble.restore({"version": CHECKPOINT_VERSION + 1})
    with pytest.raises(ValueError, match="version"):
        Ensemble.restore({})
