"""The device arithmetic the parity bar rests on: FP64 division and square root
correctly rounded (compared with the host's IEEE-754 results), and the
approximate reciprocal of the decision fast path within 4 ulp."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _cases(seed=0, n=1_000_000):
    rng = np.random.default_rng(seed)
    # operands and quotients stay inside [2^-900, 2^900], where the device
    # guarantees correct rounding
    a = [rng.uniform(0, 10, n), 10.0 ** rng.uniform(-130, 130, n), rng.uniform(1e-6, 2.0, n)]
    b = [rng.uniform(1e-3, 10, n), 10.0 ** rng.uniform(-130, 130, n), rng.uniform(0.5, 2.0, n)]
    # divisors and dividends a few ulp below / above powers of two
    k = rng.integers(-40, 40, n).astype(np.float64)
    j = rng.integers(1, 64, n).astype(np.float64)
    below = np.ldexp(1.0 - j * 2.0 ** -53, k.astype(int))
    above = np.ldexp(1.0 + j * 2.0 ** -52, k.astype(int))
    a += [rng.uniform(0.01, 10, n), below, above]
    b += [below, rng.uniform(0.01, 10, n), above[::-1]]
    # the quotient observed to be misrounded by the plain hardware sequence
    a.append(np.array([0.3499999999999998]))
    b.append(np.array([0.12499999999999993]))
    return np.concatenate(a), np.concatenate(b)


def test_division_and_sqrt_correctly_rounded(torch):
    from paper_2003_09145_amd import binding as B
    a, b = _cases()
    # near-exact squares: x = RN(s^2) +- j ulp
    rng = np.random.default_rng(1)
    s0 = rng.uniform(0.5, 4.0, 500_000)
    x2 = s0 * s0
    x2 = np.concatenate([np.nextafter(x2, np.inf), np.nextafter(x2, -np.inf), x2])
    a = np.concatenate([a, x2])
    b = np.concatenate([b, rng.permutation(x2)])
    ad = torch.from_numpy(a).cuda()
    bd = torch.from_numpy(b).cuda()
    q, q2, s, r, qp, sp = B.selftest_arith(ad, bd, plain=True)
    torch.cuda.synchronize()
    q, q2, s, r = q.cpu().numpy(), q2.cpu().numpy(), s.cpu().numpy(), r.cpu().numpy()
    qp, sp = qp.cpu().numpy(), sp.cpu().numpy()
    with np.errstate(all="ignore"):
        qe, se, re_ = a / b, np.sqrt(a), 1.0 / b
    bad_q = np.nonzero(q != qe)[0]
    bad_q2 = np.nonzero(q2 != qe)[0]
    bad_s = np.nonzero(s != se)[0]
    # the compiler's plain a / b and sqrt on the same operands: how often
    # they differ from IEEE-754 is what the correction layer is for
    bad_qp = np.nonzero(qp != qe)[0]
    bad_sp = np.nonzero(sp != se)[0]
    print(f"[arith] {len(a)} operands: div mismatches {len(bad_q)}, reciprocal-route div "
          f"mismatches {len(bad_q2)}, sqrt mismatches {len(bad_s)}; uncorrected compiler "
          f"a / b mismatches {len(bad_qp)}, sqrt mismatches {len(bad_sp)}", flush=True)
    for i in list(bad_qp[:3]) + list(bad_sp[:3]):
        print("   plain", repr(a[i]), repr(b[i]), repr(qp[i]), repr(qe[i]), repr(sp[i]),
              repr(se[i]), flush=True)
    for i in list(bad_q[:5]) + list(bad_q2[:5]):
        print("   div", repr(a[i]), repr(b[i]), repr(q[i]), repr(q2[i]), repr(qe[i]))
    assert len(bad_q) == 0 and len(bad_q2) == 0 and len(bad_s) == 0
    ulps = np.abs(r - re_) / np.spacing(np.abs(re_))
    print(f"[arith] approximate reciprocal: max error {ulps.max():.2f} ulp")
    assert ulps.max() <= 4.0
