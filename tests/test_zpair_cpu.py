"""Host model of the lazy z update of the CG passes (FP32, FP64, complex128 kernels).

CG's iterate is z = sum_j a_j p_j.  The step kernel keeps the directions in
two buffers (p_j in buffer 1 + (j & 1)), the step sizes in a two-entry ring
(a_j in a_pair[j & 1], written when iteration j's second pass ends) and adds
to z only in the first pass of even iterations j >= 2, both pending terms at
once: a_{j-2} p_{j-2} (read from the buffer that pass overwrites with p_j)
and a_{j-1} p_{j-1}.  After an even number J of iterations a fold pass adds
a_{J-2} p_{J-2}; the consumer (the CGNE start, or the complex outer phase)
then adds the last term a_{J-1} p_{J-1} from buffer 1 + ((J-1) & 1), and
reads z only when J >= 2.  This model replays that schedule with exact
rational arithmetic and random directions and checks, for every J, that the
consumer sees exactly sum_j a_j p_j, that no direction is read after it was
overwritten, and that the fold runs exactly when J is even.
"""
import random
from fractions import Fraction

import pytest


def replay(J, rng, n=3):
    bufs = {1: None, 2: None}                # buffer -> (iteration index, vector)
    z = None                                   # None: z not written yet
    a_pair = [None, None]
    dirs, steps = [], []
    for j in range(J):
        p = [Fraction(rng.randint(-9, 9), rng.randint(1, 9)) for _ in range(n)]
        a = Fraction(rng.randint(1, 9), rng.randint(1, 9))
        dirs.append(p)
        steps.append(a)
        # first pass of iteration j
        out = 1 + (j & 1)
        old = 1 + ((j + 1) & 1)
        if j >= 2 and j % 2 == 0:
            q_idx, q = bufs[out]                 # p_{j-2}, read before the overwrite
            o_idx, po = bufs[old]                # p_{j-1}
            assert (q_idx, o_idx) == (j - 2, j - 1)
            a2, a1 = a_pair[j & 1], a_pair[(j - 1) & 1]
            assert (a2, a1) == (steps[j - 2], steps[j - 1])
            base = z if j >= 4 else [Fraction(0)] * n
            assert (z is not None) == (j >= 4)
            z = [zi + a2 * qi + a1 * pi for zi, qi, pi in zip(base, q, po)]
        bufs[out] = (j, p)
        # second pass of iteration j ends: the finalize records a_j
        a_pair[j & 1] = a
    folded = False
    if J >= 2 and J % 2 == 0:                    # the fold pass
        q_idx, q = bufs[1 + (J & 1)]
        assert q_idx == J - 2
        a2 = a_pair[J & 1]
        assert a2 == steps[J - 2]
        base = z if J >= 4 else [Fraction(0)] * n
        assert (z is not None) == (J >= 4)
        z = [zi + a2 * qi for zi, qi in zip(base, q)]
        folded = True
    # the consumer: z (if J >= 2) + a_{J-1} p_{J-1}
    h_idx, ph = bufs[1 + ((J - 1) & 1)]
    assert h_idx == J - 1
    base = z if J >= 2 else [Fraction(0)] * n
    assert (z is not None) == (J >= 2)
    final = [zi + steps[J - 1] * pi for zi, pi in zip(base, ph)]
    exact = [sum(steps[j] * dirs[j][i] for j in range(J)) for i in range(n)]
    return final, exact, folded


@pytest.mark.parametrize("J", list(range(1, 14)))
def test_lazy_paired_update_gives_the_cg_iterate(J):
    rng = random.Random(J)
    for _ in range(5):
        final, exact, folded = replay(J, rng)
        assert final == exact
        assert folded == (J >= 2 and J % 2 == 0)
