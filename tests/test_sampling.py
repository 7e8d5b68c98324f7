"""The neighbourhood trick the full-size GPU tests rely on, checked on the CPU:
one step of a site computed by the oracle on its gathered 3x3x3 neighbourhood
(as a 3^3 lattice) equals the step computed on the whole lattice."""
import numpy as np

from inputs import random_state
from test_gpu_fullsize import cube


def test_cube_neighbourhood_reproduces_full_lattice_step(oracle_mod):
    N = 9
    for m, s in ((1.0, 0.0), (2.0, 1.0)):
        p = oracle_mod.params(N=N, m=m, s_early=s, s_late=s)
        p3 = dict(p, N=3)  # same eta_ref: it was fixed by the big lattice's size
        st = random_state(N, seed=61)
        sites = np.array([0, 8, 80, 81, 364, 728, 400])
        full = oracle_mod.step_sites(p, st, 4, sites)
        for k, site in enumerate(sites):
            mini = np.ascontiguousarray(st[:, cube(N, int(site))])
            got = oracle_mod.step_sites(p3, mini, 4, [13])[0]
            assert np.array_equal(got, full[k]), (m, s, site)
