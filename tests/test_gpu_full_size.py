"""Full-size checks (through the C ABI) at the benchmark's sizes and at the
largest states one GPU holds, on outputs computable one by one or on
properties that hold at any size.

  * QFT of a basis state |x> at 28 qubits (the headline size, same entry
    point): psi[k] = exp(+2 pi i x k / N) / sqrt(N) (the closed form the
    oracle is pinned to), on 4096 sampled indices and the norm.
    Tolerance: complex64 |sqrt(N) psi[k] - exp(...)| <= 2e-5 (420 gates of
    ~6e-8 rounding each on a unit-modulus value, as a random walk, plus the
    FP32 phase tables), complex128 <= 1e-11.
  * QFT of a basis state at 33 qubits complex64 (64 GiB) and 32 qubits
    complex128 (64 GiB), the largest states one GPU holds, with a random x
    whose top bits are set, so every ladder phase runs on indices above 32
    bits: the same closed form on 4096 sampled amplitudes gathered on the
    device (torch owns the memory).  Tolerance: the 28-qubit bound scaled by
    sqrt(G / 420) for G gates (complex64), 1e-11 (complex128).
  * The headline workload's own input: QFT of the seeded 28-qubit Gaussian
    state against sqrt(N) ifft (a library FFT), element by element:
    complex128 <= 1e-12 absolute per amplitude, complex64 relative L2 error
    <= 1e-5.
  * The deep random circuit generator (U3 layers and CZ matchings) at 24
    qubits and the full depth 40 (1440 gates) against the oracle: fused
    with dense blocks on and off, and one gate per launch, both dtypes
    (complex128 <= 1e-12 absolute per amplitude, complex64 relative L2 <=
    1e-5 sqrt(G / 500)).
  * The same generator at its full size (30 qubits, depth 40, complex64,
    8 GiB): fused against one gate per launch on the GPU, over the whole
    vector (relative L2 <= 2 x the complex64 amplitude bound, each side
    being within it of the exact state), on 4096 sampled amplitudes, and on
    <Z_a Z_b> / <X_a X_b> expectations (<= 1e-5).
  * The 20-qubit gradient (8 layers, 641 circuits, 200 terms,
    complex64): sampled components against the oracle's shifted energies
    (g_i = [E(theta + pi/2 e_i) - E(theta - pi/2 e_i)] / 2), <= 1e-5.
"""
import math
import os

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


@pytest.mark.parametrize("dtype,tol", [(C64, 2e-5), (C128, 1e-11)])
def test_qft28_basis_state_sampled_closed_form(sv, dtype, tol):
    n = 28
    N = 1 << n
    x = 0x9E3779B & (N - 1)
    b = I.CircuitBuilder(n)
    for q in range(n):
        if (x >> (n - 1 - q)) & 1:  # qubit q is index bit n - 1 - q
            b.add(I.X, [q])
    with sv.Context(0) as ctx:
        st = ctx.alloc(n, dtype)
        st.apply(b.build(0))
        st.qft()
        assert abs(st.norm2() - 1.0) <= (1e-5 if dtype == C64 else 1e-12)
        psi = st.get_amplitudes()
        st.free()
    rng = np.random.default_rng(11)
    ks = np.concatenate([[0, 1, N - 1, N // 2], rng.integers(0, N, 4092)])
    # exact phase x k / N mod 1 in integer arithmetic
    turns = ((x * ks) % N).astype(np.float64) / N
    want = np.exp(2j * math.pi * turns)
    got = psi[ks].astype(np.complex128) * math.sqrt(N)
    assert np.max(np.abs(got - want)) <= tol


def _basis_prep(n, x):
    b = I.CircuitBuilder(n)
    for q in range(n):
        if (x >> (n - 1 - q)) & 1:  # qubit q is index bit n - 1 - q
            b.add(I.X, [q])
    return b.build(0)


@pytest.mark.parametrize("n,dtype", [(33, C64), (32, C128)])
def test_qft_basis_state_at_the_largest_sizes(sv, n, dtype):
    import torch
    N = 1 << n
    rng = np.random.default_rng(400 + n)
    x = int(rng.integers(0, N)) | (1 << (n - 1)) | (1 << (n - 2)) | 1
    gates = n * (n + 1) // 2 + n // 2
    tol = 2e-5 * math.sqrt(gates / 420.0) if dtype == C64 else 1e-11
    ks = np.concatenate([[0, 1, N - 1, N // 2, (1 << 32) - 1, 1 << 32 if n > 32 else 3],
                         rng.integers(0, N, 4090)]).astype(np.int64)
    print(f"[full-size] qft basis n={n} dtype={dtype} x={x:#x}", flush=True)
    with sv.Context(0) as ctx:
        # torch's own work runs on its stream, the library's on the
        # context's: order them by synchronising in between
        t = torch.empty(N, dtype=torch.complex64 if dtype == C64 else torch.complex128, device="cuda")
        torch.cuda.synchronize()
        st = sv.State.from_torch(ctx, t)
        st.reset()
        st.apply(_basis_prep(n, x))
        st.qft()
        nn = st.norm2()
        ctx.synchronize()
        got = t[torch.from_numpy(ks).to("cuda")].cpu().numpy().astype(np.complex128) * math.sqrt(N)
        st.free()
        del t
        torch.cuda.empty_cache()
    assert abs(nn - 1.0) <= (1e-5 if dtype == C64 else 1e-12)
    # exact phase x k / N mod 1 in integer arithmetic (x k needs > 64 bits)
    turns = np.array([((x * int(k)) % N) / N for k in ks])
    want = np.exp(2j * math.pi * turns)
    err = np.max(np.abs(got - want))
    assert err <= tol, err


@pytest.mark.parametrize("dtype", [C64, C128])
def test_qft28_headline_input_vs_inverse_dft(sv, dtype):
    import scipy.fft
    n = 28
    N = 1 << n
    print(f"[full-size] qft28 gaussian dtype={dtype}", flush=True)
    psi = I.gaussian_state(n, 2)
    want = scipy.fft.ifft(psi, workers=min(16, os.cpu_count() or 1)) * math.sqrt(N)
    with sv.Context(0) as ctx:
        st = ctx.alloc(n, dtype)
        st.set_amplitudes(psi)
        st.qft()
        got = st.get_amplitudes()
        st.free()
    if dtype == C128:
        err = np.max(np.abs(got - want))
        assert err <= 1e-12, err
    else:
        err = _rel_l2(got, want)
        assert err <= 1e-5, err


def _rel_l2(got, want, chunk=1 << 24):
    num = den = 0.0
    for i in range(0, got.size, chunk):
        g = got[i:i + chunk].astype(np.complex128)
        w = want[i:i + chunk].astype(np.complex128)
        num += float(np.sum(np.abs(g - w) ** 2))
        den += float(np.sum(np.abs(w) ** 2))
    return math.sqrt(num / den)


@pytest.fixture(scope="module")
def deep24():
    c = I.deep_random_circuit(24, 40, 4)
    print("[full-size] deep24 oracle", flush=True)
    return c, oracle.run_circuit(c)


@pytest.mark.parametrize("dtype", [C64, C128])
@pytest.mark.parametrize("mode", ["fused_dense", "fused_no_dense", "unfused"])
def test_deep_random_24q_depth40_vs_oracle(sv, deep24, mode, dtype):
    c, want = deep24
    G = len(c.gates)
    assert G == 40 * (24 + 12)
    print(f"[full-size] deep24 {mode} dtype={dtype}", flush=True)
    kw = {"dense_fuse": -1} if mode == "fused_no_dense" else {"dense_fuse": 1}
    with sv.Context(0, **kw) as ctx:
        st = ctx.alloc(24, dtype)
        st.apply(c, flags=sv.FLAG_UNFUSED if mode == "unfused" else 0)
        got = st.get_amplitudes()
        st.free()
    if dtype == C128:
        err = np.max(np.abs(got.astype(np.complex128) - want))
        assert err <= 1e-12, err
    else:
        err = _rel_l2(got, want)
        assert err <= 1e-5 * math.sqrt(G / 500.0), err


def test_deep_random_30q_fused_vs_unfused(sv):
    n = 30
    c = I.deep_random_circuit(n, 40, 4)
    G = len(c.gates)
    rng = np.random.default_rng(30)
    pairs = [tuple(int(v) for v in rng.choice(n, 2, replace=False)) for _ in range(4)]
    terms = []
    for a, b in pairs:
        for P in "ZX":
            s = ["I"] * n
            s[a] = s[b] = P
            terms.append((1.0, "".join(s)))
    ham = I.PauliSum.from_strings(n, terms)
    ks = rng.integers(0, 1 << n, 4096)
    out = {}
    with sv.Context(0) as ctx:
        for mode in ("fused", "unfused"):
            print(f"[full-size] deep30 {mode}", flush=True)
            st = ctx.alloc(n, C64)
            st.apply(c, flags=sv.FLAG_UNFUSED if mode == "unfused" else 0)
            _, vals = st.expectation(ham, terms=True)
            out[mode] = (st.get_amplitudes(), vals)
            st.free()
    (af, vf), (au, vu) = out["fused"], out["unfused"]
    err = _rel_l2(af, au)
    assert err <= 2e-5 * math.sqrt(G / 500.0), err
    # sampled amplitudes, scaled to unit mean modulus: the largest of 4096
    # deviations whose root mean square is within the bound above stays
    # within 5 times that bound
    sq = math.sqrt(1 << n)
    samp = np.max(np.abs(af[ks].astype(np.complex128) - au[ks].astype(np.complex128))) * sq
    assert samp <= 5 * 2e-5 * math.sqrt(G / 500.0), samp
    assert np.max(np.abs(vf - vu)) <= 1e-5, (vf, vu)


def test_20q_641_circuit_gradient_sampled_components(sv):
    n = 20
    c = I.hea_circuit(n, 8)
    ham = I.random_2local(n, 200, 3)
    params = I.uniform_params(c.n_params, 3)
    with sv.Context(0) as ctx:
        e, g = ctx.param_shift_grad(c, params, ham, C64)
    assert abs(e - oracle.circuit_energy(c, params, ham)) <= 1e-5
    for i in (0, 157, c.n_params - 1):
        tp = params.copy()
        tp[i] += math.pi / 2
        tm = params.copy()
        tm[i] -= math.pi / 2
        gi = 0.5 * (oracle.circuit_energy(c, tp, ham) - oracle.circuit_energy(c, tm, ham))
        assert abs(g[i] - gi) <= 1e-5, (i, g[i], gi)
