"""The oracle's pins catch plausible mistakes.  Each case plants one mistake
in an oracle function (a dropped factor, a wrong sign, a real part for an
imaginary one, a transpose for a conjugate transpose, a wrong index or
direction) by monkeypatching it, then runs the pins that guard that
function: at least one of them must fail.  The mistakes live only in this
test's patched copies, on the CPU."""
import numpy as np
import pytest

import test_oracle_chempot as t_chempot
import test_oracle_dense as t_dense
import test_oracle_dos as t_dos
import test_oracle_hermitian as t_herm
import test_oracle_poles as t_poles
import test_oracle_symbolic as t_symb
from oracle import chempot, dense, dos, fermi, hermitian, poles, symbolic
from paper_1405_0194_amd import lattice


def _chain():
    s = lattice.config_system(0)
    H, S = s.dense()
    eig = dense.gen_eigh(H, S)
    mu = dense.half_filling_mu(eig[0])
    return s, H, S, eig, mu


def _some_pin_fails(pins):
    for fn, args in pins:
        try:
            fn(*args)
        except Exception:       # an assertion, or a numerical error the mistake causes
            return True
    return False


def _mutations():
    """(name, module, attribute, mutated-function factory, pins)."""
    ch = ("chain",)     # placeholder: replaced by the chain fixture value at run time
    return [
        ("fermi without the spin factor 2", fermi, "fermi",
         lambda f: (lambda x, beta: 0.5 * f(x, beta)),
         [(t_poles.test_fermi_closed_forms, ()), (t_poles.test_special_values_and_particle_hole_symmetry, ())]),
        ("conjugated pole weights", poles, "pole_table",
         lambda f: (lambda *a, **k: (lambda t: (t[0], {g: np.conj(w) for g, w in t[1].items()}))(f(*a, **k))),
         [(t_poles.test_rho_expansion_absolute_levels, ()), (t_poles.test_expansion_error_decays_geometrically,
                                                              ("rho",))]),
        ("shifts without mu", poles, "pole_table",
         lambda f: (lambda beta, dE, mu, P, **k: (lambda t: (t[0] - mu, t[1]))(f(beta, dE, mu, P, **k))),
         # mu must sit inside a band for the Fermi level to matter: the
         # Newton-root and Hermitian Fermi-Dirac pins put it there
         [(t_dense.test_pole_density_matrix_within_expansion_error_of_fermi_dirac, ch),
          (t_chempot.test_newton_root_matches_fermi_dirac_within_expansion_error, (0.37,)),
          (t_herm.test_close_to_fermi_dirac_within_expansion_error, ())]),
        ("real part instead of imaginary part in the pole sum", dense, "gamma_route_a",
         lambda f: (lambda H, S, shifts, weights: {
             g: np.real(sum(om[l] * dense.shifted_inverse(H, S, w) for l, w in enumerate(shifts)))
             for g, om in weights.items()}),
         [(t_dense.test_route_a_equals_route_b, ch)]),
        ("H + wS instead of H - wS", dense, "shifted_inverse",
         lambda f: (lambda H, S, w: f(H, -S, w)),
         [(t_dense.test_two_by_two_inverse_closed_form, ()), (t_dense.test_diagonal_pencil_closed_form, ()),
          (t_dense.test_route_a_equals_route_b, ch)]),
        ("trace over the lower triangle only", dense, "traces",
         lambda f: (lambda G, H, S: (float(np.sum(np.tril(G * S))), float(np.sum(np.tril(G * H))))),
         [(t_dense.test_traces_and_electron_count, ch)]),
        ("inertia counts eigenvalues above the shift", dense, "inertia_count",
         lambda f: (lambda ev, shift: len(ev) - f(ev, shift)),
         [(t_dense.test_inertia_on_pencil_with_known_spectrum, ())]),
        ("transpose instead of conjugate transpose (Hermitian)", hermitian, "gamma_route_a",
         lambda f: (lambda H, S, shifts, weights: {
             g: (a - a.T) / 2j for g, a in
             {g: sum(om[l] * dense.shifted_inverse(H, S, w) for l, w in enumerate(shifts))
              for g, om in weights.items()}.items()}),
         [(t_herm.test_routes_agree_and_are_hermitian, (1,))]),
        ("DOS bins without the spin factor", dos, "dos_bins",
         lambda f: (lambda ev, edges: 0.5 * f(ev, edges)),
         [(t_dos.test_bins_integrate_to_electron_count, ())]),
        ("LDOS at eps - i eta", dos, "ldos_dense",
         lambda f: (lambda H, S, eps, eta: f(H, S, eps, -eta)),
         [(t_dos.test_ldos_routes_agree_and_trace_is_broadened_dos, (0.13, 1e-3))]),
        # (f -> 1 - f in the boundary terms telescopes away: not a mistake)
        ("smeared count with the slope term's sign flipped", chempot, "_int_fermi1",
         lambda f: (lambda x, beta: -f(x, beta)),
         [(t_chempot.test_dense_samples_reproduce_smeared_count, ()),
          (t_chempot.test_zero_temperature_limit_is_linear_interpolation, ())]),
        ("etree parent off by one", symbolic, "etree",
         lambda f: (lambda L: (lambda p: np.where(p >= 0, np.minimum(p + 1, len(p) - 1), p))(np.asarray(f(L)))),
         [(t_symb.test_tridiagonal_no_fill_chain_etree, ()), (t_symb.test_matches_numeric_cholesky_pattern, ())]),
        ("free-energy occupation with the wrong sign", fermi, "free_occ",
         lambda f: (lambda x, beta: -f(x, beta)),
         [(t_poles.test_energy_and_derivative_sets_match_closed_forms, ()), (t_poles.test_fermi_closed_forms, ())]),
        ("Jacobi functions with m and 1 - m swapped", poles, "jacobi_complex",
         lambda f: (lambda a, b, m, m1: f(a, b, m1, m)),
         [(t_poles.test_jacobi_complex_identities, (0.3,)), (t_poles.test_jacobi_imaginary_transformation, ())]),
        ("rational function with conjugated weights", poles, "rational",
         lambda f: (lambda eps, shifts, weight: f(eps, shifts, np.conj(weight))),
         [(t_dense.test_traces_and_electron_count, ch), (t_poles.test_rho_expansion_absolute_levels, ())]),
        ("mu-derivative occupation without beta", fermi, "dfermi_dmu",
         lambda f: (lambda x, beta: f(x, beta) / beta),
         [(t_poles.test_energy_and_derivative_sets_match_closed_forms, ()), (t_poles.test_fermi_closed_forms, ())]),
        ("eigenbasis route with C transposed", dense, "gamma_route_b",
         lambda f: (lambda H, S, shifts, weights, eig=None: (lambda e: {
             g: (e[1].T * poles.rational(e[0], shifts, om)[None, :]) @ e[1] for g, om in weights.items()})(
                 dense.gen_eigh(H, S) if eig is None else eig)),
         [(t_dense.test_route_a_equals_route_b, ch)]),
        ("Hermitian trace without the transpose", hermitian, "traces",
         lambda f: (lambda G, H, S: (float(np.real(np.sum(G * S))), float(np.real(np.sum(G * H))))),
         [(t_herm.test_routes_agree_and_are_hermitian, (1,))]),
        ("broadened DOS without 2/pi", dos, "broadened_dos",
         lambda f: (lambda eig, eps, eta: f(eig, eps, eta) * (np.pi / 2.0)),
         [(t_dos.test_ldos_routes_agree_and_trace_is_broadened_dos, (0.13, 1e-3)),
          (t_dos.test_broadened_dos_tends_to_bin_counts, ())]),
        ("permutation applied as its inverse", symbolic, "permute",
         lambda f: (lambda P, perm: f(P, np.argsort(perm))),
         [(t_symb.test_permute_is_the_permutation_similarity, ())]),
        ("permutation applied to the rows only", symbolic, "permute",
         lambda f: (lambda P, perm: P[perm]),
         [(t_symb.test_permute_is_the_permutation_similarity, ()),
          (t_symb.test_permute_reversed_arrow_fills_completely, ())]),
        ("symbolic factor without fill", symbolic, "fill_pattern",
         lambda f: (lambda P: (lambda L: (np.fill_diagonal(L, True), L)[1])(np.tril(P.copy()))),
         [(t_symb.test_matches_numeric_cholesky_pattern, ()), (t_symb.test_arrow_matrices, ())]),
    ]


_CASES = _mutations()


@pytest.fixture(scope="module")
def chain():
    return _chain()


@pytest.mark.parametrize("idx", range(len(_CASES)), ids=[c[0] for c in _CASES])
def test_planted_mistake_is_caught(idx, chain, monkeypatch):
    name, mod, attr, make, pins = _CASES[idx]
    orig = getattr(mod, attr)
    monkeypatch.setattr(mod, attr, make(orig))
    pins = [(fn, (chain,) if args == ("chain",) else args) for fn, args in pins]
    assert _some_pin_fails(pins), f"no pin caught: {name}"


def test_unmutated_pins_pass(chain):
    """The same pins pass on the oracle as it stands (so the failures above
    come from the planted mistakes)."""
    seen = set()
    for name, mod, attr, make, pins in _CASES:
        for fn, args in pins:
            key = (fn.__name__, args)
            if key in seen:
                continue
            seen.add(key)
            fn(*((chain,) if args == ("chain",) else args))
