"""GPU path (through the C ABI) vs the FP64 oracle, element by element.

Tolerances (stated, not tuned per case):
  complex128 amplitudes: <= 1e-12 absolute per amplitude
  complex64 amplitudes:  relative L2 error <= 1e-5 * max(1, sqrt(G / 500))
                         (G = gates; one rounding of ~6e-8 per gate and
                         component accumulates as a random walk)
  energies / gradients:  complex128 <= 1e-10, complex64 <= 1e-5 absolute
"""
import math

import numpy as np
import pytest

import oracle
from paper_2512_23183_amd import inputs as I

pytestmark = pytest.mark.gpu

C64, C128 = 0, 1


@pytest.fixture(scope="module")
def sv():
    from paper_2512_23183_amd import sv as svmod
    return svmod


@pytest.fixture(scope="module")
def ctx(sv):
    c = sv.Context(0)
    yield c
    c.close()


def amp_tol_ok(got, want, dtype, n_gates):
    got = got.astype(np.complex128)
    if dtype == C128:
        err = np.max(np.abs(got - want)) if want.size else 0.0
        return err <= 1e-12, err
    rel = np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)
    return rel <= 1e-5 * max(1.0, math.sqrt(n_gates / 500.0)), rel


def run_gpu(ctx, circuit, params, psi0, dtype, flags=0):
    st = ctx.alloc(circuit.n, dtype)
    st.set_amplitudes(psi0)
    st.apply(circuit, params, flags)
    out = st.get_amplitudes()
    st.free()
    return out


def single_gate(n, kind, qs, ang, mat=None):
    b = I.CircuitBuilder(n)
    if kind in (I.MAT1, I.MAT2):
        b.add_matrix(qs, mat)
    else:
        b.add(kind, qs, angles=ang)
    return b.build()


def operand_sets(n, arity, rng):
    if arity == 1:
        return [[q] for q in range(n)]
    if arity == 2:
        s = [[0, n - 1], [n - 1, 0], [n // 2, n // 2 + 1], [1, 0], [n - 2, n - 1]]
        s += [list(map(int, rng.choice(n, 2, replace=False))) for _ in range(3)]
        return s
    s = [[0, 1, n - 1], [n - 1, n - 2, 0], [n // 2, 0, n - 1]]
    s += [list(map(int, rng.choice(n, 3, replace=False))) for _ in range(3)]
    return s


@pytest.mark.parametrize("dtype", [C128, C64])
@pytest.mark.parametrize("n", [5, 11, 15])
@pytest.mark.parametrize("kind", sorted(I.KIND_NAMES))
def test_each_kind_every_position(ctx, kind, n, dtype):
    rng = np.random.default_rng(1000 + 31 * kind + n)
    psi0 = I.gaussian_state(n, 7 + n)
    for qs in operand_sets(n, I.ARITY[kind], rng):
        ang = list(rng.uniform(0, 2 * math.pi, 3))
        mat = None
        if kind in (I.MAT1, I.MAT2):
            d = 2 if kind == I.MAT1 else 4
            z = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
            mat, _ = np.linalg.qr(z)
        c = single_gate(n, kind, qs, ang, mat)
        want = oracle.run_circuit(c, None, psi0)
        for flags in (0, 1):
            got = run_gpu(ctx, c, None, psi0, dtype, flags)
            ok, err = amp_tol_ok(got, want, dtype, 1)
            assert ok, (I.KIND_NAMES[kind], qs, flags, err)


@pytest.mark.parametrize("dtype", [C128, C64])
@pytest.mark.parametrize("n,steps", [(10, 12), (15, 6)])
def test_trotter_xyz_evolution_vs_oracle(ctx, n, steps, dtype):
    # XX / YY / ZZ rotations and time-dependent Z fields from |1...1>, then
    # the energy under H(t) at the final time
    t = 1.2
    c = I.trotter_xyz_circuit(n, steps, t)
    want = oracle.run_circuit(c)
    ham = I.xyz_chain(n, h=I.xyz_field(t))
    e_ref, _ = oracle.energy(want, ham)
    for flags in (0, 1):
        st = ctx.alloc(n, dtype)
        st.apply(c, None, flags)
        got = st.get_amplitudes()
        e = st.expectation(ham)
        st.free()
        ok, err = amp_tol_ok(got, want, dtype, c.n_gates)
        assert ok, (flags, err)
        assert abs(e - e_ref) <= (1e-10 if dtype == C128 else 1e-5), (flags, e, e_ref)


@pytest.mark.parametrize("dtype", [C128, C64])
def test_sweeps_on_far_apart_bits(ctx, dtype):
    # one launch per gate on a 24-qubit state: index sets 32 MiB and more
    # apart (several work items per thread), in-wavefront partners (lane
    # shuffles), bit 0 pairs, controls above and below the wavefront span
    n = 24
    psi0 = I.gaussian_state(n, 77)
    rng = np.random.default_rng(5)
    z = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    m2, _ = np.linalg.qr(z)
    cases = [(I.U3, [0], [0.3, 1.2, 2.1]), (I.U3, [1], [0.5, 0.1, 0.9]), (I.H, [2], []),
             (I.CNOT, [0, 1], []), (I.CNOT, [1, 0], []), (I.CNOT, [0, n - 1], []), (I.CNOT, [0, n - 3], []),
             (I.CRY, [n - 1, 0], [0.7]), (I.X, [n - 5], []), (I.RY, [n - 7], [1.3]),
             (I.SWAP, [0, 2], []), (I.SWAP, [1, n - 1], []), (I.CZ, [0, 1], []), (I.CP, [0, n - 2], [0.4]),
             (I.RZZ, [0, 1], [0.8]), (I.MAT2, [1, 0], None)]
    for kind, qs, ang in cases:
        c = single_gate(n, kind, qs, ang, m2 if kind == I.MAT2 else None)
        want = oracle.run_circuit(c, None, psi0)
        got = run_gpu(ctx, c, None, psi0, dtype, 1)
        ok, err = amp_tol_ok(got, want, dtype, 1)
        assert ok, (I.KIND_NAMES[kind], qs, err)


@pytest.mark.parametrize("dtype", [C128, C64])
@pytest.mark.parametrize("n,G,seed", [(1, 20, 1), (2, 40, 2), (8, 300, 3), (13, 300, 4),
                                      (14, 300, 5), (17, 300, 6), (20, 200, 7)])
def test_random_circuits(ctx, n, G, seed, dtype):
    c = I.random_circuit(n, G, seed, n_params=7)
    params = I.uniform_params(c.n_params, seed)
    psi0 = I.gaussian_state(n, seed)
    want = oracle.run_circuit(c, params, psi0)
    for flags in (0, 1):
        got = run_gpu(ctx, c, params, psi0, dtype, flags)
        ok, err = amp_tol_ok(got, want, dtype, G)
        assert ok, (flags, err)


def test_empty_circuit_is_identity(ctx):
    c = I.CircuitBuilder(6).build()
    psi0 = I.gaussian_state(6, 3)
    np.testing.assert_array_equal(run_gpu(ctx, c, None, psi0, C128), psi0)


@pytest.mark.parametrize("dtype", [C128, C64])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 12, 13, 16, 20])
def test_qft_vs_oracle_and_inverse_dft(ctx, n, dtype):
    psi0 = I.gaussian_state(n, 2)
    want = oracle.qft(psi0)
    ref = math.sqrt(1 << n) * np.fft.ifft(psi0)
    G = n + n * (n - 1) // 2 + n // 2
    for flags in (0, 1):
        st = ctx.alloc(n, dtype)
        st.set_amplitudes(psi0)
        st.qft(flags)
        got = st.get_amplitudes()
        st.free()
        ok, err = amp_tol_ok(got, want, dtype, G)
        assert ok, (flags, err)
        if dtype == C128:
            assert np.max(np.abs(got - ref)) <= 1e-12


@pytest.mark.parametrize("dtype", [C128, C64])
@pytest.mark.parametrize("n,T,seed", [(3, 10, 1), (10, 27, 2), (16, 200, 3), (20, 60, 4)])
def test_expectation_vs_oracle(ctx, n, T, seed, dtype):
    ham = I.xyz_chain(n) if T == 27 else I.random_2local(n, T, seed)
    psi = I.gaussian_state(n, seed)
    e_ref, _ = oracle.energy(psi, ham)
    st = ctx.alloc(n, dtype)
    st.set_amplitudes(psi)
    e, tv = st.expectation(ham, terms=True)
    assert abs(e - e_ref) <= (1e-10 if dtype == C128 else 1e-5), (e, e_ref)
    for t in range(0, ham.n_terms, max(1, ham.n_terms // 7)):
        r = oracle.pauli_expectation(psi, ham.strings()[t]).real
        assert abs(tv[t] - r) <= (1e-10 if dtype == C128 else 1e-5)
    assert abs(st.norm2() - 1.0) <= (1e-12 if dtype == C128 else 1e-6)
    st.free()


def _mixed_pauli_sum(n, seed, n_random, n_diag):
    """Random strings of every weight (X/Y supports up to the full width),
    one X/Y support shared by 32 terms of every Y parity, and n_diag Z-only
    strings (more than one expectation pass holds)."""
    rng = np.random.default_rng(seed)
    terms = []
    for _ in range(n_random):
        w = int(rng.integers(1, n + 1))
        s = ["I"] * n
        for q in rng.choice(n, w, replace=False):
            s[q] = "XYZ"[int(rng.integers(0, 3))]
        terms.append((float(rng.normal()), "".join(s)))
    for a in "XY":
        for b in "XY":
            for zpat in range(8):
                s = ["I"] * n
                s[0], s[n - 1] = a, b
                for i, q in enumerate((1, 2, n - 2)):
                    if (zpat >> i) & 1:
                        s[q] = "Z"
                terms.append((float(rng.normal()), "".join(s)))
    seen = set()
    while len(seen) < n_diag:
        z = int(rng.integers(1, 1 << n))
        if z in seen:
            continue
        seen.add(z)
        terms.append((float(rng.normal()) * 0.01,
                      "".join("Z" if (z >> q) & 1 else "I" for q in range(n))))
    order = rng.permutation(len(terms))
    # coefficients scaled to sum |c_t| = 50: one rounding of the state to
    # complex64 (relative 2^-24 per component, |delta| <= 2^-24 |psi|) then
    # moves the energy by at most 2 |delta| sum |c_t| = 6e-6, inside the flat
    # complex64 tolerance of 1e-5
    scale = 50.0 / sum(abs(c) for c, _ in terms)
    return I.PauliSum.from_strings(n, [(terms[i][0] * scale, terms[i][1]) for i in order])


@pytest.mark.parametrize("bits", [0, 6, 9])
@pytest.mark.parametrize("n", [7, 12])
def test_expectation_widths_supports_and_many_terms(sv, n, bits):
    # tile widths from 6 bits (wide supports go to the HBM pair pass) to the
    # default; > 1024 diagonal terms split the diagonal group across passes
    ham = _mixed_pauli_sum(n, 100 + n + bits, 120, min(1100, (1 << n) - 1))
    psi = I.gaussian_state(n, 7 + bits)
    strings = ham.strings()
    ref = np.array([oracle.pauli_expectation(psi, s).real for s in strings])
    e_ref = float(np.dot(ham.coeffs, ref))
    c = sv.Context(0, expect_bits_c64=bits, expect_bits_c128=bits)
    try:
        for dtype, tol in ((C128, 1e-10), (C64, 1e-5)):
            st = c.alloc(n, dtype)
            st.set_amplitudes(psi)
            e, tv = st.expectation(ham, terms=True)
            st.free()
            assert abs(e - e_ref) <= tol, (dtype, e, e_ref)
            assert np.max(np.abs(tv - ref)) <= tol, dtype
    finally:
        c.close()


def test_batched_gradient_narrow_expectation_tiles(sv):
    # the multi-pass batched path with several expectation passes per circuit
    n = 14
    circ = I.hea_circuit(n, 1)
    params = I.uniform_params(circ.n_params, 21)
    ham = _mixed_pauli_sum(n, 22, 40, 30)
    e_ref, g_ref = oracle.param_shift(circ, params, ham)
    c = sv.Context(0, expect_bits_c64=7, expect_bits_c128=7)
    try:
        for dtype, tol in ((C128, 1e-10), (C64, 1e-5)):
            e, g = c.param_shift_grad(circ, params, ham, dtype)
            assert abs(e - e_ref) <= tol
            assert np.max(np.abs(g - g_ref)) <= tol
    finally:
        c.close()


def test_expectation_renormalises(ctx):
    n = 9
    ham = I.random_2local(n, 40, 5)
    psi = I.gaussian_state(n, 5)
    e_ref, _ = oracle.energy(psi, ham)
    st = ctx.alloc(n, C128)
    st.set_amplitudes(3.0 * psi)
    assert abs(st.expectation(ham) - e_ref) <= 1e-12
    st.normalize()
    assert abs(st.norm2() - 1.0) <= 1e-13
    st.free()


def test_empty_hamiltonian(ctx):
    st = ctx.alloc(4, C128)
    ham = I.PauliSum(4, np.zeros(0), np.zeros((0, 4), dtype=np.uint8))
    assert st.expectation(ham) == 0.0
    st.free()


def test_nonfinite_state_reports_enumeric(ctx, sv):
    st = ctx.alloc(3, C128)
    psi = np.zeros(8, dtype=complex)
    psi[0] = np.nan
    st.set_amplitudes(psi)
    with pytest.raises(sv.SvError) as e:
        st.expectation(I.xyz_chain(3))
    assert e.value.name == "SV_ENUMERIC"
    st.free()


# ---------------------------------------------------------------------------
# Parameter-shift gradients
# ---------------------------------------------------------------------------

def test_psr_10q_xyz_chain_c128(ctx):
    n = 10
    c = I.hea_circuit(n, 4)
    ham = I.xyz_chain(n)
    params = I.uniform_params(c.n_params, 1)
    e_ref, g_ref = oracle.param_shift(c, params, ham)
    e, g = ctx.param_shift_grad(c, params, ham, C128)
    assert abs(e - e_ref) <= 1e-10
    assert np.max(np.abs(g - g_ref)) <= 1e-10
    e64, g64 = ctx.param_shift_grad(c, params, ham, C64)
    assert abs(e64 - e_ref) <= 1e-5
    assert np.max(np.abs(g64 - g_ref)) <= 1e-5


@pytest.mark.parametrize("flags", [2, 3])
def test_psr_plain_paths_match(ctx, flags):
    n = 8
    c = I.hea_circuit(n, 2)
    ham = I.xyz_chain(n)
    params = I.uniform_params(c.n_params, 4)
    e_ref, g_ref = oracle.param_shift(c, params, ham)
    e, g = ctx.param_shift_grad(c, params, ham, C128, flags)
    assert abs(e - e_ref) <= 1e-10
    assert np.max(np.abs(g - g_ref)) <= 1e-10


def _app_d_rows():
    from tests.test_oracle_pins import _app_d_table, _half_ulp, _theta
    return _app_d_table(), _half_ulp, _theta


@pytest.mark.parametrize("case", list(I.APP_D_CASES))
def test_psr_app_d_table_on_gpu(ctx, case):
    table, half_ulp, theta = _app_d_rows()
    th_tok, g_tok = table[case]
    params = np.array([theta(t) for t in th_tok])
    c, ham = I.app_d_circuit(), I.app_d_observable()
    _, g = ctx.param_shift_grad(c, params, ham, C128)
    _, g_ref = oracle.param_shift(c, params, ham)
    assert np.max(np.abs(g - g_ref)) <= 1e-12
    for j in range(4):
        assert abs(g[j] - float(g_tok[j])) <= half_ulp(g_tok[j])


def test_psr_every_angle_kind_shared_params(ctx):
    kinds = [I.RX, I.RY, I.RZ, I.U3, I.CP, I.CRX, I.CRY, I.CRZ, I.RXX, I.RYY,
             I.RZZ, I.CNOT, I.H, I.CZ, I.SWAP]
    c = I.random_circuit(5, 60, 41, kinds=kinds, n_params=6)
    ham = I.random_2local(5, 20, 42)
    params = I.uniform_params(c.n_params, 43)
    e_ref, g_ref = oracle.param_shift(c, params, ham)
    e, g = ctx.param_shift_grad(c, params, ham, C128)
    assert abs(e - e_ref) <= 1e-10
    assert np.max(np.abs(g - g_ref)) <= 1e-10


@pytest.mark.parametrize("dtype", [C128, C64])
def test_psr_multipass_circuits(ctx, dtype):
    # states larger than one workgroup's LDS take the pass executor
    n = 15
    c = I.hea_circuit(n, 1)
    ham = I.random_2local(n, 30, 8)
    params = I.uniform_params(c.n_params, 9)
    e_ref, g_ref = oracle.param_shift(c, params, ham)
    e, g = ctx.param_shift_grad(c, params, ham, dtype)
    tol = 1e-10 if dtype == C128 else 1e-5
    assert abs(e - e_ref) <= tol
    assert np.max(np.abs(g - g_ref)) <= tol


def test_psr_ansatz_random_2local_small_c64(ctx):
    # the 20-qubit gradient's structure (RY/RZ + ladder, random 2-local) at a size the
    # oracle finishes quickly
    n = 12
    c = I.hea_circuit(n, 2)
    ham = I.random_2local(n, 200, 3)
    params = I.uniform_params(c.n_params, 3)
    e_ref, g_ref = oracle.param_shift(c, params, ham)
    e, g = ctx.param_shift_grad(c, params, ham, C64)
    assert abs(e - e_ref) <= 1e-5
    assert np.max(np.abs(g - g_ref)) <= 1e-5


def test_batch_energies_mixed_sizes(ctx):
    ns = [1, 3, 8, 12, 13, 14, 16]
    circs, prms, hams, refs = [], [], [], []
    for i, n in enumerate(ns):
        c = I.hea_circuit(n, 2)
        p = I.uniform_params(c.n_params, 50 + i)
        h = I.random_2local(n, 25, 60 + i) if n >= 2 else I.PauliSum.from_strings(1, [(0.7, "Z"), (0.2, "X")])
        circs.append(c)
        prms.append(p)
        hams.append(h)
        refs.append(oracle.circuit_energy(c, p, h))
    for dtype, tol in ((C128, 1e-10), (C64, 1e-5)):
        e = ctx.batch_energies(circs, prms, hams, dtype)
        assert np.max(np.abs(e - np.array(refs))) <= tol


def test_invalid_gradient_args(ctx, sv):
    c = I.hea_circuit(4, 1)
    with pytest.raises(sv.SvError) as e:
        ctx.param_shift_grad(c, np.zeros(3), I.xyz_chain(4), C128)
    assert e.value.name == "SV_EINVAL"
    with pytest.raises(sv.SvError) as e:
        ctx.param_shift_grad(c, np.zeros(8), I.xyz_chain(5), C128)
    assert e.value.name == "SV_EINVAL"


def test_torch_tensor_as_state(ctx, sv):
    import torch
    n = 10
    psi0 = I.gaussian_state(n, 12)
    t = torch.from_numpy(psi0.copy()).to("cuda:0")
    torch.cuda.synchronize()
    st = sv.State.from_torch(ctx, t)
    c = I.hea_circuit(n, 1)
    p = I.uniform_params(c.n_params, 1)
    st.apply(c, p)
    ctx.synchronize()
    got = t.cpu().numpy()
    want = oracle.run_circuit(c, p, psi0)
    assert np.max(np.abs(got - want)) <= 1e-12
    st.free()


def test_autotune_picks_valid_widths_and_caches(sv, tmp_path):
    cache = str(tmp_path / "tune.txt")
    c = sv.Context(0)
    try:
        first = c.autotune(C64, 14, cache)
        assert 11 <= first["tile_bits_c64"] <= 14 and 11 <= first["expect_bits_c64"] <= 14
        assert 11 <= first["tile_bits_layers_c64"] <= 14
        assert 10 <= first["perm_bits_c64"] <= 12
        assert first["dense_fuse"] in (1, -1)
        lines = open(cache).read().splitlines()
        assert len(lines) == 1 and "dtype0 n14" in lines[0] and " dense=" in lines[0] and " layers=" in lines[0]
        second = c.autotune(C64, 14, cache)        # cache hit: same widths, no new line
        assert second == first
        assert len(open(cache).read().splitlines()) == 1
        tuned = c.autotune(C128, 13)
        assert 9 <= tuned["tile_bits_c128"] <= 12 and 9 <= tuned["tile_bits_layers_c128"] <= 12
        # the tuned context still matches the oracle
        n = 14
        circ = I.random_circuit(n, 120, 31, n_params=4)
        params = I.uniform_params(circ.n_params, 32)
        psi0 = I.gaussian_state(n, 33)
        want = oracle.run_circuit(circ, params, psi0)
        for dtype in (C64, C128):
            got = run_gpu(c, circ, params, psi0, dtype)
            ok, err = amp_tol_ok(got, want, dtype, circ.n_gates)
            assert ok, (dtype, err)
    finally:
        c.close()


@pytest.mark.parametrize("n,depth", [(9, 4), (14, 3), (17, 2)])
@pytest.mark.parametrize("kind", ["trotter", "deep"])
def test_dense_mfma_blocks_match_oracle(sv, n, depth, kind):
    # complex64 runs of fixed gates on four qubits that include a two-qubit
    # rotation (the XYZ Trotter circuit's RXX / RYY / RZZ) become dense
    # 16x16 blocks on MFMA; layers of U3 and CZ (one-qubit gates and
    # diagonals only) stay with the four-bit register stages either way
    if kind == "trotter":
        circ = I.trotter_xyz_circuit(n, depth, 0.7)
    else:
        circ = I.deep_random_circuit(n, depth, 40 + n)
    psi0 = I.gaussian_state(n, 41 + n)
    want = oracle.run_circuit(circ, None, psi0)
    for fuse in (1, -1):
        c = sv.Context(0, dense_fuse=fuse)
        try:
            got = run_gpu(c, circ, None, psi0, C64)
        finally:
            c.close()
        ok, err = amp_tol_ok(got, want, C64, circ.n_gates)
        assert ok, (fuse, err)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_forced_dense_blocks_of_each_width_match_oracle(sv, k):
    # dense_fuse = k: every run of at least two fixed gates on at most k
    # qubits becomes a dense block (padded to four qubits, MFMA), here on
    # layers of U3 and CZ, which the default policy leaves to the register
    # stages; 14 qubits (several tiles per pass), depth 6
    n = 14
    circ = I.deep_random_circuit(n, 6, 70 + k)
    assert sv.plan_info(circ, dtype=C64, dense_fuse=k)["dense_blocks"] > 0
    psi0 = I.gaussian_state(n, 71 + k)
    want = oracle.run_circuit(circ, None, psi0)
    c = sv.Context(0, dense_fuse=k)
    try:
        got = run_gpu(c, circ, None, psi0, C64)
    finally:
        c.close()
    ok, err = amp_tol_ok(got, want, C64, circ.n_gates)
    assert ok, (k, err)
