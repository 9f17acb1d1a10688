"""GPU: the frugal rejection sampler (qflex_frugal_sample) against the oracle, element by
element: accepted values bit for bit (both sides decide u * M < N p in FP64 with the same
roundings), the error estimate to 1e-12 relative (FP64 sums in different orders)."""
import numpy as np
import pytest

import rqc_inputs as R
from oracle import sampling as S
from oracle import statevector as E1
from paper_1811_09599_amd import build_grid, fidelity_samples, frugal_sample

pytestmark = pytest.mark.gpu


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(*a):
    print(*a, flush=True)


def _run(amps, order, u, n_q, m):
    import torch
    acc, tail = frugal_sample(torch.from_numpy(amps).cuda(), torch.from_numpy(order).cuda(),
                              torch.from_numpy(u).cuda(), n_q, m)
    return acc.cpu().numpy().tolist(), tail


@pytest.mark.parametrize("nb,blen,nc,m", [(3000, 64, 64, 10.0), (3000, 64, 7, 3.0),
                                          (1000, 256, 100, 10.0), (513, 64, 1, 1.5),
                                          (5, 4096, 300, 10.0)])
def test_sampler_matches_oracle_on_porter_thomas_batches(nb, blen, nc, m):
    _need_gpu()
    _say("frugal sampler", nb, blen, nc, m)
    n_q = 30
    amps = R.porter_thomas_amplitudes(nb, blen, n_q, 100 + nc)
    order, u = R.sampling_draws(nb, blen, nc, 200 + nc)
    got, tail = _run(amps, order, u, n_q, m)
    assert got == S.frugal_sample(amps, order, u, n_q, m)
    want = S.tail_error(amps, n_q, m)
    assert abs(tail - want) <= 1e-12 * want
    assert any(g >= 0 for g in got)


def test_sampler_edge_cases():
    _need_gpu()
    import torch
    _say("frugal sampler edge cases")
    n_q = 8
    amps = R.porter_thomas_amplitudes(40, 16, n_q, 3)
    order, u = R.sampling_draws(40, 16, 16, 4)
    # no visits: nothing accepted, the estimate still covers every amplitude
    got, tail = _run(amps, order[:, :0].copy(), u[:, :0].copy(), n_q, 10.0)
    assert got == [-1] * 40
    assert abs(tail - S.tail_error(amps, n_q, 10.0)) <= 1e-12 * max(tail, 1e-300)
    # no batches
    acc, tail = frugal_sample(torch.zeros((0, 16), dtype=torch.complex128, device="cuda"),
                              torch.zeros((0, 3), dtype=torch.int32, device="cuda"),
                              torch.zeros((0, 3), dtype=torch.float64, device="cuda"), n_q)
    assert acc.numel() == 0 and tail == 0.0
    # huge probabilities: the first visit always accepts; zeros: never
    big = np.full((40, 16), np.sqrt(20.0 / 2 ** n_q), dtype=complex)
    got, tail = _run(big, order, u, n_q, 10.0)
    assert got == order[:, 0].tolist() and abs(tail - 20.0) < 1e-12
    got, _ = _run(np.zeros((40, 16), dtype=complex), order, u, n_q, 10.0)
    assert got == [-1] * 40
    # a value outside the batch marks its batch and the binding refuses the result
    bad = order.copy()
    bad[7, 3] = 16
    with pytest.raises(ValueError):
        _run(amps, bad, u, n_q, 10.0)


def test_sampler_on_contracted_open_batches():
    """End to end: 4x4 RQC amplitudes with a 4-qubit open batch (16 values per closed
    bit-string) from the contraction, sampled on the device; the oracle takes the same
    amplitudes (bit-exact decisions) and the state vector's own amplitudes (decisions agree
    except where u * M and N p nearly tie)."""
    _need_gpu()
    import torch
    _say("frugal sampler on 4x4 open batches")
    c = R.grid_rqc(4, 4, 16, 1000)
    op = [12, 13, 14, 15]
    bits = R.bitstrings(16, 400, 1500, op)
    g = build_grid(c, open_qubits=op)
    amps = g.contract_amplitudes(bits, device=True)
    order, u = R.sampling_draws(400, 16, 16, 1700)
    acc, tail = frugal_sample(amps, torch.from_numpy(order).cuda(), torch.from_numpy(u).cuda(),
                              16, 10.0)
    acc = acc.cpu().numpy().tolist()
    a_host = amps.cpu().numpy()
    assert acc == S.frugal_sample(a_host, order, u, 16, 10.0)
    assert abs(tail - S.tail_error(a_host, 16, 10.0)) <= 1e-12 * tail
    ref = E1.amplitudes(c, bits, op)
    assert np.max(np.abs(a_host - ref)) * 2 ** 8 < 1e-5
    same = np.mean(np.array(acc) == np.array(S.frugal_sample(ref, order, u, 16, 10.0)))
    assert same >= 0.99
    # at depth 16 the 4x4 output is close to Porter-Thomas: acceptance near 1 - 0.9^16
    rate = np.mean(np.array(acc) >= 0)
    assert abs(rate - S.batch_acceptance(10.0, 16)) < 0.1
    g.close()


def test_fidelity_samples_match_oracle():
    """Fidelity-f samples of a 4x4 RQC with a 4-qubit open batch: the device path contracts only
    the exact batches; the oracle composes the same coins, draws and uniform bit-strings with
    the device's amplitudes (bit-exact) and with the state vector's (agreement but for ties)."""
    _need_gpu()
    import torch  # noqa: F401
    _say("fidelity-f samples, 4x4")
    c = R.grid_rqc(4, 4, 16, 1001)
    op = [12, 13, 14, 15]
    nb, f = 600, 0.3
    closed = R.bitstrings(16, nb, 1600, op)
    uniform = R.bitstrings(16, nb, 1601)
    rng = np.random.Generator(np.random.PCG64(1602))
    coins = rng.random(nb)
    order, u = R.sampling_draws(nb, 16, 16, 1603)
    g = build_grid(c, open_qubits=op)
    samples, status = fidelity_samples(g, closed, coins, uniform, order, u, f)
    exact = coins < f
    assert np.array_equal(status != 0, exact)
    dev_amps = np.zeros((nb, 16), dtype=complex)
    dev_amps[exact] = g.contract_amplitudes(closed[exact]).cpu().numpy()
    ref_s, ref_st = S.fidelity_samples(dev_amps, closed, op, coins, uniform, order, u, 16, 10.0, f)
    assert status.tolist() == ref_st
    for b in range(nb):
        if ref_st[b] != -1:
            assert samples[b].tolist() == ref_s[b]
    sv = E1.amplitudes(c, closed, op)
    _, sv_st = S.fidelity_samples(sv, closed, op, coins, uniform, order, u, 16, 10.0, f)
    assert np.mean(np.array(sv_st) == status) >= 0.99
    # rows of another width than the circuit's are refused before any call (the library
    # reads n_qubits bytes per batch)
    with pytest.raises(ValueError, match="closed_bits"):
        fidelity_samples(g, closed[:, :15], coins, uniform[:, :15], order, u, f)
    g.close()


def test_fidelity_samples_checks_arguments_before_any_launch():
    """An order value outside the open batch in an exact batch, a fidelity outside [0, 1] or a
    grid of several circuits is rejected on the host; the same value in a batch that is not
    exact is never read.  No batch at all returns empty results."""
    from paper_1811_09599_amd import _ffi as F

    _need_gpu()
    _say("fidelity-f samples: argument checks")
    c = R.grid_rqc(4, 4, 16, 1001)
    op = [12, 13, 14, 15]
    g = build_grid(c, open_qubits=op)
    closed = R.bitstrings(16, 4, 1700, op)
    uniform = R.bitstrings(16, 4, 1701)
    order, u = R.sampling_draws(4, 16, 16, 1702)
    coins = np.array([0.1, 0.9, 0.1, 0.9])
    bad = order.copy()
    bad[1, 3] = 16  # batch 1 is not exact at f = 0.5: never read
    samples, status = fidelity_samples(g, closed, coins, uniform, bad, u, 0.5)
    assert status[1] == 0 and samples[1].tolist() == uniform[1].tolist()
    bad[0, 3] = 16  # batch 0 is exact
    with pytest.raises(F.QflexError) as e:
        fidelity_samples(g, closed, coins, uniform, bad, u, 0.5)
    assert e.value.status == F.E_INVALID
    with pytest.raises(F.QflexError):
        fidelity_samples(g, closed, coins, uniform, order, u, 1.5)
    s0, st0 = fidelity_samples(g, closed[:0], coins[:0], uniform[:0], order[:0], u[:0], 0.5)
    assert s0.shape == (0, 16) and st0.shape == (0,)
    g.close()
    g2 = build_grid([c, c], open_qubits=op)
    with pytest.raises(F.QflexError):
        fidelity_samples(g2, closed, coins, uniform, order, u, 0.5)
    g2.close()
