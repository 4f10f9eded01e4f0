"""GPU: FP64 source iterations whose inputs are all non-negative tag each
flux of the data-driven sweep by its sign bit (alternating between the
sweeps that fill one level-position array) instead of writing empty markers
for the next sweep; any negative input switches the solve back to markers.
On one graph, a sequence that crosses between the two kinds of sweep in
both directions, with odd and even sweep counts (so both tags meet stale
values of the other), warm starts with and without negative fluxes, and
plain sweeps in between: every result against the oracle's, within 1e-12
(bit-identical in practice)."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import J, dev, gpu_graph, host, need_gpu, rel_max

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,k", [("tetcheck16_s8", 3), ("delaunay_s4", 1), ("hex3_cyclic", 0)])
def test_tagged_and_marker_solves_alternate(oracle_mod, name, k):
    need_gpu()
    if k == 0:
        p = W.Problem("hex3cyc", W.hex_lattice(3, 0.3, 1), *W.quadrature(8, 3),
                      np.full(27, 1.3), np.full(27, 0.9), np.ones(27))
    else:
        p = W.config(k, "small") if k == 3 else W.config(k)
    print(f"[case] {name} cells={p.n_cells} dirs={p.n_dirs}", flush=True)
    og = oracle_mod.graph_for(p)
    gg = gpu_graph(p)
    rng = np.random.default_rng(7)
    q_pos = p.q
    q_neg = p.q - 1.5 * rng.random(p.n_cells)       # some cells with a negative source
    assert (q_neg < 0).any()
    # (source, boundary inflow, iterations): non-negative (tagged), negative
    # source (markers), negative inflow (markers), then tagged again with odd
    # and even counts
    steps = [(q_pos, 0.0, 5), (q_neg, 0.0, 4), (q_pos, 0.3, 3), (q_pos, -0.2, 2), (q_pos, 0.0, 4), (q_pos, 0.1, 7)]
    for i, (q, psi_b, iters) in enumerate(steps):
        psi_ref, phi_ref, _ = og.source_iteration(p.sigma_t, p.sigma_s, q, p.weight, iters, psi_b=psi_b)
        phi = dev(np.zeros(p.n_cells))
        psi = dev(np.zeros((p.n_dirs, p.n_cells)))
        J.solve(gg, dev(p.sigma_t), dev(p.sigma_s), dev(q), phi, psi, psi_boundary=psi_b, mode=J.JSWEEP_FP64,
                tol=0.0, max_iter=iters, allow_not_converged=True)
        e1, e2 = rel_max(host(phi), phi_ref), rel_max(host(psi), psi_ref)
        print(f"[tags {name}] step {i} ({'negative' if (q < 0).any() or psi_b < 0 else 'non-negative'} inputs, "
              f"{iters} sweeps): phi {e1:.2e} psi {e2:.2e} bitexact {np.array_equal(host(psi), psi_ref)}", flush=True)
        assert e1 <= 1e-12 and e2 <= 1e-12, i
        if i in (0, 3):
            # plain sweeps in between (markers): after the tagged solve of
            # step 0 first the one that allocates nothing (it fills the
            # array with markers itself), then the ordinary one
            if i == 0:
                out = dev(np.zeros((p.n_dirs, p.n_cells)))
                J.jsweep_sweep_noalloc(gg, dev(p.sigma_t), dev(q), out)
                assert np.array_equal(host(out), og.sweep(p.sigma_t, q)), i
            out = dev(np.zeros((p.n_dirs, p.n_cells)))
            J.sweep(gg, dev(p.sigma_t), dev(q), out)
            assert np.array_equal(host(out), og.sweep(p.sigma_t, q)), i
    gg.close()


def test_warm_start_with_negative_fluxes(oracle_mod):
    """A warm start from fluxes with negative entries: the solve uses
    markers; one from the previous non-negative solve's fluxes is tagged.
    Both continue the oracle's iteration exactly."""
    need_gpu()
    p = W.config(3, "small")
    og = oracle_mod.graph_for(p)
    gg = gpu_graph(p)
    psi_ref, phi_ref, _ = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 6)
    psi5, _, _ = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 5)
    for label, start in (("non-negative", psi5), ("with negative entries", None)):
        if start is None:
            # every seventh cell's fluxes negated in every direction: their
            # phi, and so the next sweep's source there, is negative, and
            # the solve writes markers
            start = psi5.copy()
            start[:, ::7] *= -1.0
        phi = dev(np.zeros(p.n_cells))
        psi = dev(start)
        J.solve(gg, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, psi, mode=J.JSWEEP_FP64 | J.JSWEEP_WARM_START,
                tol=0.0, max_iter=1, allow_not_converged=True)
        # one sweep from `start`: phi_start = sum_m w psi, source q + sigma_s phi_start
        phi_start = np.einsum("m,mk->k", p.weight, start)
        src = p.q + p.sigma_s * phi_start
        want = og.sweep(p.sigma_t, src)
        e = rel_max(host(psi), want)
        print(f"[tags warm] start {label}: psi after one sweep {e:.2e}", flush=True)
        assert e <= 1e-12, label
        if label == "non-negative":
            assert rel_max(host(psi), psi_ref) <= 1e-12
    gg.close()


def test_negative_zero_inputs_keep_their_sign(oracle_mod):
    """A source, scattering cross section and boundary inflow of -0.0 make
    every flux -0.0 in the oracle's arithmetic.  A sign-tagged store would
    not keep that sign, so the solve takes markers and returns the oracle's
    bits, the sign of every zero included."""
    need_gpu()
    p = W.config(3, "small")
    og = oracle_mod.graph_for(p)
    gg = gpu_graph(p)
    q = np.full(p.n_cells, -0.0)
    sigma_s = np.full(p.n_cells, -0.0)
    psi_ref, phi_ref, _ = og.source_iteration(p.sigma_t, sigma_s, q, p.weight, 3, psi_b=-0.0)
    assert np.signbit(psi_ref).all() and (psi_ref == 0.0).all()
    phi = dev(np.ones(p.n_cells))
    psi = dev(np.ones((p.n_dirs, p.n_cells)))
    J.solve(gg, dev(p.sigma_t), dev(sigma_s), dev(q), phi, psi, psi_boundary=-0.0, mode=J.JSWEEP_FP64, tol=0.0,
            max_iter=3, allow_not_converged=True)
    got, got_phi = host(psi), host(phi)
    print(f"[tags -0] psi sign bits set: {np.signbit(got).mean():.3f} (oracle {np.signbit(psi_ref).mean():.3f})",
          flush=True)
    assert np.array_equal(np.signbit(got), np.signbit(psi_ref)) and np.array_equal(got, psi_ref)
    assert np.array_equal(np.signbit(got_phi), np.signbit(phi_ref)) and np.array_equal(got_phi, phi_ref)
    # the next solve with non-negative inputs on the same graph is tagged again
    psi_ref2, phi_ref2, _ = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 3)
    J.solve(gg, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, psi, mode=J.JSWEEP_FP64, tol=0.0, max_iter=3,
            allow_not_converged=True)
    assert rel_max(host(psi), psi_ref2) <= 1e-12 and rel_max(host(phi), phi_ref2) <= 1e-12
    gg.close()
