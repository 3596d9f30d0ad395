"""The pins constrain the oracle: deliberately wrong copies of it fail them.

Each mutant is the oracle source with one plausible mistake planted in it
(a sign, a neighbour taken on the wrong side, a dropped factor, a wrong
opposite direction, ...).  It is compiled into a temporary library and the
fast CPU pins run against it in a subprocess (HMCSC_ORACLE_LIB).  Every mutant
must make at least one pin fail; the unmodified source must pass the same
pins.  Nothing here touches the GPU library or the repository's built oracle.
"""
import os
import subprocess
import sys

import pytest

from oracle import ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")
PINS = ["test_oracle_forces.py", "test_oracle_closed_forms.py", "test_oracle_invariants.py",
        "test_oracle_lattice.py", "test_oracle_shear_wave.py", "test_oracle_brinkman.py", "test_oracle_guo.py",
        "test_oracle_pressure.py"]

# (name, text in hmcsc_oracle.c, replacement, which occurrence (1-based))
MUTANTS = [
    ("cohesion sign", "Finter[a] = -rho_s[s] * p->G * g[a];", "Finter[a] = rho_s[s] * p->G * g[a];", 1),
    ("adhesion sign", "Fads[a] = -rho_s[s] * p->G_ads[s] * g[a];", "Fads[a] = rho_s[s] * p->G_ads[s] * g[a];", 1),
    ("cohesion neighbour at x - c_i", "wrap(x + L->c[i][0], p->nx), wrap(y + L->c[i][1], p->ny),",
     "wrap(x - L->c[i][0], p->nx), wrap(y - L->c[i][1], p->ny),", 1),
    ("adhesion neighbour at x - c_i", "wrap(x + L->c[i][0], p->nx), wrap(y + L->c[i][1], p->ny),",
     "wrap(x - L->c[i][0], p->nx), wrap(y - L->c[i][1], p->ny),", 2),
    ("streaming to x - c_i", "wrap(x + L->c[i][0], p->nx), wrap(y + L->c[i][1], p->ny),",
     "wrap(x - L->c[i][0], p->nx), wrap(y - L->c[i][1], p->ny),", 3),
    ("external force not split by density", "rho_s[s] / rho * p->F_ext[a]", "p->F_ext[a]", 1),
    ("bounce-back without the opposite direction", "nsx * fl[s][L->opp[i]]", "nsx * fl[s][i]", 1),
    ("relaxation not weighted by 1 - n_s", "- (1.0 - nsx) / p->tau[s] * (fl[s][i] - feq)",
     "- 1.0 / p->tau[s] * (fl[s][i] - feq)", 1),
    ("bounce-back blend without 1 - n_s", "post[s][i] = (1.0 - nsx) * fl[s][i]", "post[s][i] = fl[s][i]", 1),
    ("relaxation time off by one half", "- (1.0 - nsx) / p->tau[s] * (fl[s][i] - feq)",
     "- (1.0 - nsx) / (p->tau[s] + 0.5) * (fl[s][i] - feq)", 1),
    ("second-order term of the equilibrium doubled", "(cu * cu) / (2.0 * CS2 * CS2)", "(cu * cu) / (CS2 * CS2)", 1),
    ("velocity term of the equilibrium halved", "1.0 + cu / CS2", "1.0 + cu / (2.0 * CS2)", 1),
    ("force shift without tau", "p->tau[s] * Ft[s][a] / rho_s[s]", "Ft[s][a] / rho_s[s]", 1),
    ("common velocity not tau-weighted", "num[a] += j[s][a] / p->tau[s];", "num[a] += j[s][a];", 1),
    ("macroscopic velocity without the half force", "(js + Ft[s][a] / 2.0)", "(js + Ft[s][a])", 1),
    ("adhesion reads component 0's n_s field", "const double s_nb = ns_at(p, ns, s, nb);",
     "const double s_nb = ns_at(p, ns, 0, nb);", 1),
    ("pressure without the interaction term", "pr[n] = CS2 * (rho_tot + inter);", "pr[n] = CS2 * rho_tot;", 1),
    ("pressure interaction without the stencil scale", "p->g_scale * p->G * rf[n] * rf[N + n]",
     "p->G * rf[n] * rf[N + n]", 1),
    ("u_macro divided by the first component's density", "u[a * N + n] = rho_tot > 0.0 ? m / rho_tot : 0.0;",
     "u[a * N + n] = rf[n] > 0.0 ? m / rf[n] : 0.0;", 1),
    ("reservoir range closed at hi", "xyz[p->res[r].axis] < p->res[r].hi", "xyz[p->res[r].axis] <= p->res[r].hi", 1),
    ("reservoir axis ignored", "xyz[p->res[r].axis] >= p->res[r].lo && xyz[p->res[r].axis] < p->res[r].hi",
     "xyz[2] >= p->res[r].lo && xyz[2] < p->res[r].hi", 1),
    ("u_macro reads component 0's n_s field", "m += (1.0 - ns_at(p, ns, s, n)) * (js + Ft[s][a] / 2.0);",
     "m += (1.0 - ns_at(p, ns, 0, n)) * (js + Ft[s][a] / 2.0);", 1),
    ("Guo term with the first component's tau", "guo_term(L, i, p->tau[s], ueq, Ft[s])",
     "guo_term(L, i, p->tau[0], ueq, Ft[s])", 1),
    ("Guo term with the other component's force", "guo_term(L, i, p->tau[s], ueq, Ft[s])",
     "guo_term(L, i, p->tau[s], ueq, Ft[1 - s < p->ncomp ? 1 - s : 0])", 1),
    ("one n_s field for both components", "return ns[(p->c_ns == 2 ? s : 0) * ncells(p) + n];",
     "return ns[n];", 1),
    ("macroscopic velocity not weighted by 1 - n_s", "m += (1.0 - ns_at(p, ns, s, n)) * (js", "m += (js", 1),
    ("reservoirs not reset", "    reset_reservoirs(p, L, f_out);\n    return 0;", "    return 0;", 1),
    ("axis weight 1/16", "w1 = 1.0 / 18.0;", "w1 = 1.0 / 16.0;", 1),
    ("stencil scale ignored", "g[a] += p->g_scale * L->w[i] * r_nb * L->c[i][a];",
     "g[a] += L->w[i] * r_nb * L->c[i][a];", 1),
    # the GS-WBS with Guo forcing
    ("Guo term without its second-order part", "((cF - uF) / CS2 + cu * cF / (CS2 * CS2))",
     "((cF - uF) / CS2)", 1),
    ("Guo term without its velocity part", "((cF - uF) / CS2", "((cF) / CS2", 1),
    ("Guo prefactor dropped", "(1.0 - 1.0 / (2.0 * tau)) * L->w[i]", "L->w[i]", 1),
    ("Guo term not weighted by 1 - n_s", "post[s][i] += (1.0 - nsx) * guo_term(", "post[s][i] += guo_term(", 1),
    ("Guo velocity without the half force", "(j[s][a] + 0.5 * Ft[s][a])", "(j[s][a])", 1),
    ("Guo velocity not weighted by 1 - n_s", "m += (1.0 - ns_at(p, ns, s, n)) * (j[s][a]", "m += (j[s][a]", 1),
]


# Pins too slow to run against every mutant, each with a mutant it must catch:
# (name, text, replacement, occurrence, pin)
TARGETED = [
    ("macroscopic velocity not weighted by 1 - n_s, against the Buckley-Leverett pin",
     "m += (1.0 - ns_at(p, ns, s, n)) * (js", "m += (js", 1,
     "test_oracle_buckley_leverett.py::test_front_moves_with_the_buckley_leverett_shock"),
    ("adhesion halved, against the stored Washburn fronts behind the contact-angle pin",
     "Fads[a] = -rho_s[s] * p->G_ads[s] * g[a];", "Fads[a] = -0.5 * rho_s[s] * p->G_ads[s] * g[a];", 1,
     "test_oracle_washburn.py::test_stored_full_size_front_is_the_oracles"),
]


def _mutate(src: str, old: str, new: str, k: int) -> str:
    pos = -1
    for _ in range(k):
        pos = src.find(old, pos + 1)
        assert pos >= 0, f"mutation site not found: {old!r} (occurrence {k})"
    return src[:pos] + new + src[pos + len(old):]


def _run_pins(lib: str, pins=None, threads=None) -> subprocess.CompletedProcess:
    env = dict(os.environ, HMCSC_ORACLE_LIB=lib)
    if threads:
        env["OMP_NUM_THREADS"] = str(threads)
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           *[os.path.join(TESTS, f) for f in (pins or PINS)]]
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)


# The mutants are independent: they are compiled and checked four at a time
# (two OpenMP threads each, so the host is not oversubscribed), once per
# session, and each parametrized test reads its own outcome.
WORKERS, THREADS = 4, 2


def _check(tmp, key, old, new, k, pins):
    src = open(ref.SRC).read()
    tag = "".join(ch if ch.isalnum() else "_" for ch in key)[:60]
    msrc = os.path.join(tmp, f"{tag}.c")
    with open(msrc, "w") as fh:
        fh.write(_mutate(src, old, new, k) if old is not None else src)
    lib = ref.compile_to(msrc, os.path.join(tmp, f"{tag}.so"))
    r = _run_pins(lib, pins, THREADS)
    return r.returncode, r.stdout[-2000:]


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    from concurrent.futures import ThreadPoolExecutor
    tmp = str(tmp_path_factory.mktemp("mutants"))
    jobs = {("pins", "unmodified"): (None, None, 0, None)}
    for name, old, new, k in MUTANTS:
        jobs[("pins", name)] = (old, new, k, None)
    for name, old, new, k, pin in TARGETED:
        jobs[("targeted", name)] = (old, new, k, [pin])
        jobs[("targeted-unmodified", name)] = (None, None, 0, [pin])
    with ThreadPoolExecutor(WORKERS) as pool:
        futs = {key: pool.submit(_check, tmp, key[0] + key[1], *job) for key, job in jobs.items()}
        return {key: f.result() for key, f in futs.items()}


def test_unmodified_oracle_passes_the_pins(outcomes):
    rc, out = outcomes[("pins", "unmodified")]
    assert rc == 0, out


@pytest.mark.parametrize("name", [m[0] for m in MUTANTS])
def test_mutant_fails_a_pin(outcomes, name):
    rc, _ = outcomes[("pins", name)]
    assert rc != 0, f"no pin caught the mutant '{name}'"


@pytest.mark.parametrize("name", [m[0] for m in TARGETED])
def test_targeted_mutant_fails_its_pin(outcomes, name):
    pin = [m[4] for m in TARGETED if m[0] == name][0]
    rc0, out0 = outcomes[("targeted-unmodified", name)]
    assert rc0 == 0, (pin, out0)
    rc, _ = outcomes[("targeted", name)]
    assert rc != 0, f"the pin {pin} did not catch the mutant '{name}'"
