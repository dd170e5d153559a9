"""The first-derivative op tables (gen/emit_deriv.py), run on the CPU by the
same numpy interpreter as the integral tables (tests/test_t3_tables.py) and
compared with the oracle's derivative integrals, which are pinned to finite
differences and translational invariance (tests/test_oracle_deriv.py).  The
quartets are one-primitive shells, so the contraction coefficient of each is
N(alpha, l), as the primitive-quartet interface gives them."""
import numpy as np
import pytest

import oracle
import workloads
from paper_2605_10312_amd.gen import emit_deriv, emit_t3
from tests.test_t3_tables import run_tables


def _basis(ls, cen, ex):
    return workloads.Basis(l=np.array(ls, np.int32), nprim=np.ones(4, np.int32), centers=np.array(cen, float),
                           exps=np.array(ex, float), coefs=np.ones(4), atom=np.arange(4, dtype=np.int32),
                           atoms=np.array(cen, float))


@pytest.mark.parametrize("ls", [(0, 0, 0, 0), (1, 0, 0, 0), (1, 1, 0, 0), (1, 0, 1, 0), (1, 1, 1, 1), (2, 0, 0, 0),
                                (2, 1, 1, 0), (2, 2, 1, 1), (2, 1, 2, 1), (2, 2, 2, 2)])
def test_deriv_tables_match_oracle(ls):
    t = emit_deriv.build_deriv_tables(*ls)
    w = emit_t3.build_wave_tables_from(emit_deriv.build_deriv_tables(*ls, bundle=emit_t3.WAVE), ls)
    n = 3
    cen, ex = workloads.prim_quartets(max(ls), n, seed=81 + sum(ls), box=1.5, exp_range=(0.3, 3.0))
    shape = [4, 3] + [2 * l + 1 for l in ls]
    for tt, ops, K, zero in ((t, None, None, None), (w.t, w.ops, emit_t3.WAVE, w.zero)):
        got = run_tables(tt, ls, cen, ex, ops=ops, K=K, zero=zero, weights=True, shape=shape)
        for q in range(n):
            b = _basis(ls, cen[q], ex[q])
            ref = oracle.eri_deriv_shell_quartet(b, 0, 1, 2, 3, precision="long double")
            scale = np.abs(ref).max()
            err = np.abs(got[q] - ref).max()
            assert err <= 1e-12 * scale + 1e-14, (ls, q, err, scale)
    print(f"{ls}: {t.nslots} slots, {t.n_vrr} + {t.n_p2} ops, LDS {w.lds_bytes} B")
