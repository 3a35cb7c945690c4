"""The library's average-atom pseudopotential (arche_aa_pseudopotential, host
code) against the oracle's (Sec. 2.4): the form-factor table, Delta E_AA, the
chemical potential and the pseudo-density's coefficients.  No GPU."""
import math

import numpy as np
import pytest

from oracle import aa
from paper_2606_13283_amd import arche
from paper_2606_13283_amd import workloads as W


@pytest.mark.parametrize("T_ev,frac,xc", [(10.0, 0.6, True), (100.0, 0.5, False)])
def test_library_matches_oracle(T_ev, frac, xc):
    rho = 1.0 / W.cell_length(1, 2.7) ** 3
    kT = W.ev(T_ev)
    tab_o, dE_o, d = aa.pseudopotential(13.0, rho, kT, frac, xc=xc, dq=0.01, n_q=120)
    tab_l, res = arche.aa_pseudopotential(13.0, rho, kT, frac, xc=xc, dq=0.01, n_q=120)
    P = d["pseudo"]
    assert abs(res["r_cut"] - P.r_cut) <= 1e-14 * P.r_cut
    assert abs(res["mu"] - d["aa"].mu) <= 1e-10 * abs(d["aa"].mu)
    for k in ("a", "b", "c"):
        assert abs(res[k] - getattr(P, k)) <= 1e-8 * max(abs(getattr(P, k)), 1.0), k
    assert np.max(np.abs(tab_l - tab_o)) <= 1e-9 * np.max(np.abs(tab_o))
    assert abs(res["dE_AA"] - dE_o) <= 1e-9 * abs(dE_o)


def test_library_rejects_bad_parameters():
    for kw in (dict(Z=-1.0), dict(r_cut_frac=1.0), dict(kT=0.0)):
        args = dict(Z=13.0, rho_ion=0.01, kT=0.3, r_cut_frac=0.5)
        args.update(kw)
        with pytest.raises(arche.ArcheError):
            arche.aa_pseudopotential(**args)
