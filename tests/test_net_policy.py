"""Host logic of the learned setup's evaluation (no GPU): the plain setup's
role as fallback and judge of the network-initialised setup."""
import pytest

from paper_2111_05012_amd.train_net import choose_setup, summarize


def _row(net_iters, plain_iters, net_conv=True, plain_conv=True, net_error=False):
    def ent(it, conv):
        return dict(setup_s=0.01, iters=it, relres=1e-11 if conv else 1e-6, converged=conv, solve_s=0.02)
    n = ent(net_iters, net_conv)
    if net_error:
        n = dict(setup_s=None, iters=None, relres=None, converged=False, solve_s=None, error='EINVAL')
    return dict(plain=ent(plain_iters, plain_conv), ablate=ent(plain_iters + 2, True), net=n)


def test_network_kept_when_never_worse():
    assert choose_setup([_row(5, 5), _row(4, 6)]) == 'net'


@pytest.mark.parametrize('rows', [
    [_row(5, 5), _row(7, 6)],               # more outer iterations on one seed
    [_row(4, 6, net_conv=False)],            # did not converge
    [_row(4, 6), _row(0, 6, net_error=True)],  # setup failed
    [],                                      # nothing to judge by
])
def test_plain_setup_is_the_fallback(rows):
    assert choose_setup(rows) == 'plain'


def test_summary_skips_failed_setups():
    s = summarize([_row(5, 5), _row(0, 6, net_error=True)])
    assert s['net']['runs'] == 1 and s['net']['failed'] == 1 and s['net']['iters'] == 5
    assert s['plain']['iters'] == 5.5 and s['ablate']['iters'] == 7.5
