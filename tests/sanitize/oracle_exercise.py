"""Drive every part of the oracle's C code once, small, for a run under
AddressSanitizer and UndefinedBehaviorSanitizer (started by
tests/test_sanitizers.py with ORACLE_SANITIZE_LIB set and libasan preloaded).
Prints the checks it makes; exits non-zero if one fails."""

import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402
from workloads import configs  # noqa: E402
from workloads.nuclear import synthetic_elastic_nuclear, with_elastic_nuclear  # noqa: E402


def check(cond, what):
    print(("ok   " if cond else "FAIL ") + what, flush=True)
    if not cond:
        sys.exit(1)


def balance(rec):
    b = rec[:, oracle.R_DEP] + rec[:, oracle.R_ESC] + rec[:, oracle.R_NUC] + \
        rec[:, oracle.R_TRUNC] - rec[:, oracle.R_E0]
    return float(np.abs(b).max() / rec[:, oracle.R_E0].max())


def main():
    assert os.environ.get("ORACLE_SANITIZE_LIB"), "run through tests/test_sanitizers.py"
    check(oracle.lib()._name == os.environ["ORACLE_SANITIZE_LIB"], "the sanitized build is loaded")
    wl = configs.water100_small(n=300)
    ph, p = wl.phantom, wl.params
    nt = workloads.nuclear_for_phantom(ph, p.lattice())
    zs = [z for m in ph.materials for z in m.Z]
    As = [a for m in ph.materials for a in m.A]
    nte = with_elastic_nuclear(nt, synthetic_elastic_nuclear(zs, As, p.lattice(), seed=3))
    # transport: each switch set, with and without nuclear data, records on
    for flags in (oracle.ALL, oracle.ALL | oracle.ECUT, oracle.ALL & ~oracle.SBM,
                  oracle.LOSS | oracle.EOR, oracle.LOSS | oracle.ELASTIC, 0):
        for tables in (None, nt, nte):
            r = oracle.transport(ph, wl.spots, p, tables, seed=5, flags=flags, records=True,
                                 n_threads=2)
            check(r.ledger[oracle.L_HIST] == 300 and balance(r.records) < 1e-9,
                  f"transport flags={flags} tables={'none' if tables is None else 'data'}")
    # heterogeneous phantoms, small
    for mk in (configs.slab, configs.insert, configs.ct_like):
        w = mk(100.0, n=200, size=24)
        r = oracle.transport(w.phantom, w.spots, w.params,
                             workloads.nuclear_for_phantom(w.phantom, w.params.lattice()),
                             seed=1, records=True, n_threads=2)
        d = oracle.dose(r.edep, w.phantom)
        check(np.isfinite(d).all() and balance(r.records) < 1e-9, f"{mk.__name__} transport and dose")
    # gamma, local and global
    rng = np.random.default_rng(0)
    a = rng.random((9, 8, 7)) + 0.5
    b = a * (1 + 0.01 * rng.standard_normal(a.shape))
    for local in (True, False):
        frac, ne, npass = oracle.gamma_pass_rate(a, b, (0.1, 0.1, 0.1), local=local, n_threads=2)
        check(0 <= frac <= 1 and ne == a.size, f"gamma local={local}: {frac:.3f}")
    # random numbers, source
    h = np.arange(64, dtype=np.uint64)
    words = oracle.rng_blocks(9, h, np.zeros(64, np.uint32), np.ones(64, np.uint32))
    check(words.shape == (64, 4), "Philox blocks")
    src = oracle.source(wl.spots[0], 0.0, 3, 0, 100)
    check(np.isfinite(src).all(), "source sampler")
    # physics functionals and the nuclear view
    m = ph.materials[0]
    for E in (0.06, 1.0, 50.0, 250.0):
        vals = [oracle.stopping_mass(m, E), oracle.straggle_mass(m, E), oracle.csda_range_g(m, E),
                oracle.ld_sigma(m, 1.0, E), oracle.elastic_cut(m, p, 1.0, E, flags=oracle.ECUT),
                oracle.channel_total_rate(m, p, 1.0, E, nte, flags=oracle.ALL | oracle.ECUT)]
        check(all(math.isfinite(v) for v in vals), f"functionals at {E} MeV")
    for t in (1e-5, 0.01, 0.03, 0.5):
        c, s = oracle.sbm_polar(t, rng.standard_normal(8), rng.random(8))
        check(np.isfinite(c).all() and np.isfinite(s).all(), f"SBM sampler at t={t}")
    v = oracle.NuclearView(nte)
    for E in (1.0, 60.0, 200.0):
        vals = [v.sigma_barn(0, E), v.table(0, "u", E, 0.4), v.ni_density(0, E, 0.3),
                v.ni_integral(0, E, 0.3), v.h_nuclear_density(E, 0.2),
                v.h_nuclear_antiderivative(E, 0.2),
                v.elastic_sample_mu(1, 1.008, E, 0.4), v.elastic_sample_mu(8, 16.0, E, 0.7),
                v.elastic_cum_barn(1, 1.008, E, -math.cos(0.04), 0.5)]
        check(all(math.isfinite(x) for x in vals), f"nuclear view at {E} MeV")
        u, mu = v.draw(0, E, 0.3, 0.6)
        check(math.isfinite(u) and math.isfinite(mu), f"inelastic draw at {E} MeV")
    check(math.isfinite(oracle.bspline3(np.arange(8.0), 5, -1.0, 0.4, 0.3)), "B-spline")
    print("oracle exercise done", flush=True)


if __name__ == "__main__":
    main()
