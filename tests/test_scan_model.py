"""FP64 model of the chunked-scan decomposition the IIR kernel uses, checked
against the oracle on the CPU.

This is not the oracle and shares no code with it or with the HIP path: it
restates the decomposition (per-chunk zero-state response, inclusive scan of
chunk states with powers of the 2x2 chunk transition, wave and tile
aggregates, look-back reduction over up to 64 predecessors with powers of the
tile transition, fold into the chunk-entering state, zero-input correction)
so that the algebra is verified before any kernel runs.  Sizes are scaled
down (lanes, waves, chunk length) so the python loops stay fast; the algebra
does not depend on them.
"""
import numpy as np
import pytest

from oracle import oracle as O


def _tables(coef, L, lanes, waves):
    b0, b1, b2, a1, a2 = coef
    A = np.array([[-a1, 1.0], [-a2, 0.0]])
    g = np.zeros((L, 2))
    P = np.eye(2)
    for t in range(L):
        g[t] = P[0]
        P = P @ A
    Phi = P                                       # A^L
    fold = [np.linalg.matrix_power(Phi, k) for k in range(lanes)]
    Psi = np.linalg.matrix_power(Phi, lanes)
    psi = [np.linalg.matrix_power(Psi, w) for w in range(waves)]
    PhiT = np.linalg.matrix_power(Psi, waves)
    lb = [np.linalg.matrix_power(PhiT, 2 ** j) for j in range(7)]
    apow = [np.linalg.matrix_power(A, t + 1) for t in range(L)]
    return dict(g=g, fold=fold, psi=psi, lb=lb, apow=apow)


def _zsr(coef, x):
    b0, b1, b2, a1, a2 = coef
    s1 = s2 = 0.0
    y = np.empty_like(x)
    states = np.empty((x.size, 2))
    for n, xv in enumerate(x):
        yv = b0 * xv + s1
        s1 = b1 * xv - a1 * yv + s2
        s2 = b2 * xv - a2 * yv
        y[n] = yv
        states[n] = (s1, s2)
    return y, states


def model_channel(x, sos, L, lanes, waves, rng, state_in=None):
    """Runs the decomposition over one channel; returns (y, final state)."""
    T = L * lanes * waves
    N = x.size
    nt = -(-N // T)
    xp = np.concatenate([x, np.zeros(nt * T - N)])
    v = xp.copy()
    S = len(sos)
    final = np.zeros((S, 2))
    for s, coef in enumerate(sos):
        tb = _tables(coef, L, lanes, waves)
        agg = np.zeros((nt, 2))
        inc = np.zeros((nt, 2))
        for t in range(nt):
            seg = v[t * T:(t + 1) * T].reshape(waves, lanes, L)
            y0 = np.empty_like(seg)
            z = np.empty((waves, lanes, 2))
            cap = np.empty((waves, lanes, L, 2))
            for w in range(waves):
                for ln in range(lanes):
                    y0[w, ln], st = _zsr(coef, seg[w, ln])
                    z[w, ln] = st[-1]
                    cap[w, ln] = st
            # Kogge-Stone inclusive scan inside each wave
            wsc = z.copy()
            d = 1
            while d < lanes:
                prev = wsc.copy()
                for ln in range(d, lanes):
                    wsc[:, ln] = prev[:, ln] + prev[:, ln - d] @ tb["fold"][d].T
                d *= 2
            E = np.zeros(2)
            Ew = []
            for w in range(waves):
                Ew.append(E.copy())
                E = tb["psi"][1] @ E + wsc[w, -1] if waves > 1 else tb["lb"][0] @ E + wsc[w, -1]
            # with one wave psi[1] does not exist; the tile transition is lb[0]
            agg[t] = E
            if t == 0:
                P = np.zeros(2) if state_in is None else state_in[s]
            else:
                # look-back: predecessors randomly published only their
                # aggregate; walk back in windows of 64
                P = np.zeros(2)
                M = np.eye(2)
                base = t - 1
                published_inc = rng.random(t) < 0.3
                published_inc[0] = True
                while True:
                    vals = []
                    stop = False
                    for i in range(64):
                        q = base - i
                        if q < 0:
                            break
                        if published_inc[q]:
                            vals.append(inc[q])
                            stop = True
                            break
                        vals.append(agg[q])
                    vals += [np.zeros(2)] * (64 - len(vals))
                    vv = [np.array(a) for a in vals]
                    for j in range(6):
                        dd = 2 ** j
                        vv = [vv[i] + (tb["lb"][j] @ vv[i + dd] if i + dd < 64 else 0) for i in range(64)]
                    P = P + M @ vv[0]
                    if stop:
                        break
                    M = M @ tb["lb"][6]
                    base -= 64
            inc[t] = tb["lb"][0] @ P + agg[t]
            out = np.empty_like(seg)
            for w in range(waves):
                e = Ew[w] + tb["psi"][w] @ P
                for ln in range(lanes):
                    pv = wsc[w, ln - 1] if ln > 0 else np.zeros(2)
                    si = pv + tb["fold"][ln] @ e
                    out[w, ln] = y0[w, ln] + tb["g"] @ si
                    pos = t * T + (w * lanes + ln) * L
                    if pos <= N - 1 < pos + L:
                        r = N - 1 - pos
                        final[s] = tb["apow"][r] @ si + cap[w, ln, r]
            v[t * T:(t + 1) * T] = out.reshape(-1)
    return v[:N], final


@pytest.mark.parametrize("N", [1, 7, 95, 96, 97, 500, 2000])
def test_chunked_scan_model_matches_oracle(N):
    rng = np.random.default_rng(N)
    sos = np.array([[0.2, 0.4, 0.2, -1.2, 0.5], [1.0, -1.9, 1.0, -1.97, 0.99],
                    [0.5, 0.1, -0.3, 0.3, 0.2]])
    x = rng.standard_normal(N)
    si = rng.standard_normal((3, 2))
    y, fin = model_channel(x, sos, L=4, lanes=8, waves=3, rng=rng, state_in=si)
    ref, st = O.sos(x[None], sos, state_in=si[None], return_state=True)
    assert np.max(np.abs(y - ref[0])) < 1e-10 * max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(fin - st[0])) < 1e-10 * max(1.0, np.max(np.abs(st)))


def test_chunked_scan_model_long_lookback():
    # many tiles so that the look-back crosses more than one 64-tile window
    rng = np.random.default_rng(3)
    sos = np.array([[1.0, 0.0, 0.0, -1.8, 0.9]])
    N = 8 * 150 + 3
    x = rng.standard_normal(N)
    y, _ = model_channel(x, sos, L=2, lanes=2, waves=2, rng=rng)
    ref = O.sos(x[None], sos)[0]
    assert np.max(np.abs(y - ref)) < 1e-9 * np.max(np.abs(ref))


# ------------------------------------------------ cascade-level carry

def _cascade_transition(sec):
    """One-sample transition of a cascade's free response (zero input), state
    order (s1, s2) of section 0, then section 1, ...: block (i, i) = A_i,
    block (i, j < i) = B_i (prod_{j<l<i} D_l) C, C = (1, 0), D_l = b0 of
    section l, B_i = (b1 - a1 b0, b2 - a2 b0) of section i."""
    S = len(sec)
    F = np.zeros((2 * S, 2 * S))
    for i, (b0, b1, b2, a1, a2) in enumerate(sec):
        F[2 * i:2 * i + 2, 2 * i:2 * i + 2] = [[-a1, 1.0], [-a2, 0.0]]
        B = np.array([b1 - a1 * b0, b2 - a2 * b0])
        for j in range(i):
            pr = np.prod([sec[l][0] for l in range(j + 1, i)]) if i > j + 1 else 1.0
            F[2 * i:2 * i + 2, 2 * j] = B * pr
    return F


@pytest.mark.parametrize("S", [1, 2, 5, 8])
def test_cascade_transition_is_the_free_response(S):
    # the state of the whole cascade after n samples of zero input, started
    # from an arbitrary state, is F^n times that state (run by the oracle)
    from paper_2504_08624_amd import design, signals
    sec = design.random_sections(signals.rng(71, S), S, 0.5, 0.99)
    st = signals.rng(72, S).standard_normal((1, S, 2))
    n = 300
    _, s_end = O.sos(np.zeros((1, n)), sec, state_in=st, return_state=True)
    F = _cascade_transition(sec)
    np.testing.assert_allclose(np.linalg.matrix_power(F, n) @ st.reshape(-1), s_end.reshape(-1),
                               rtol=1e-10, atol=1e-12)


def test_cascade_look_back_two_phase_equals_oracle():
    # per tile: (A) run the cascade from a zero tile-entering state -> the
    # cascade's tile aggregate E_t; (B) P_{t+1} = F^T P_t + E_t; (C) run the
    # cascade from P_t.  The outputs equal the oracle's.
    from paper_2504_08624_amd import design, signals
    S, T, ntiles = 4, 96, 7
    sec = design.random_sections(signals.rng(73), S, 0.5, 0.995)
    x = signals.rng(74).standard_normal(T * ntiles)
    FT = np.linalg.matrix_power(_cascade_transition(sec), T)
    P = np.zeros(2 * S)
    y = np.empty_like(x)
    for t in range(ntiles):
        seg = x[t * T:(t + 1) * T][None, :]
        _, E = O.sos(seg, sec, state_in=np.zeros((1, S, 2)), return_state=True)
        yt = O.sos(seg, sec, state_in=P.reshape(1, S, 2))
        y[t * T:(t + 1) * T] = yt[0]
        P = FT @ P + E.reshape(-1)
    np.testing.assert_allclose(y, O.sos(x[None, :], sec)[0], rtol=1e-9, atol=1e-12)


def test_cascade_zero_input_response_form_equals_oracle():
    # phase C as the chain kernel's table form: the tile output is the response
    # to a zero tile-entering state plus, at sample r of chunk k,
    # G[r] . (F^(L k) P) with G[r] = c F^r and c[2s] = prod_{t>s} b0_t, c[2s+1] = 0
    # (the s1 register of section s reaches the output through the b0 of every
    # later section).  Only the lower block triangle of F^(L k) is used.
    from paper_2504_08624_amd import design, signals
    S, L, chunks, ntiles = 6, 8, 12, 5
    T = L * chunks
    sec = design.random_sections(signals.rng(75), S, 0.5, 0.995)
    x = signals.rng(76).standard_normal(T * ntiles)
    F = _cascade_transition(sec)
    D = 2 * S
    c = np.zeros(D)
    for s in range(S):
        c[2 * s] = np.prod([sec[t][0] for t in range(s + 1, S)]) if s + 1 < S else 1.0
    G = np.array([c @ np.linalg.matrix_power(F, r) for r in range(L)])
    Mk = [np.linalg.matrix_power(F, L * k) for k in range(chunks)]
    lower = np.array([[j <= (i | 1) for j in range(D)] for i in range(D)])
    for m in Mk:  # the powers are block lower triangular
        assert np.all(m[~lower] == 0.0)
    FT = np.linalg.matrix_power(F, T)
    P = np.zeros(D)
    y = np.empty_like(x)
    for t in range(ntiles):
        seg = x[t * T:(t + 1) * T][None, :]
        yA, E = O.sos(seg, sec, state_in=np.zeros((1, S, 2)), return_state=True)
        n = np.arange(T)
        corr = np.array([G[i % L] @ ((Mk[i // L] * lower) @ P) for i in n])
        y[t * T:(t + 1) * T] = yA[0] + corr
        P = FT @ P + E.reshape(-1)
    np.testing.assert_allclose(y, O.sos(x[None, :], sec)[0], rtol=1e-9, atol=1e-11)


# ------------------------------------------------ matrix-core cascade form

def _cascade_io(sec):
    """Input column b and output row c of the cascade's state space (same
    state order as _cascade_transition), and its feed-through d: the output is
    c s + d x and the next state F s + b x."""
    S = len(sec)
    b = np.zeros(2 * S)
    c = np.zeros(2 * S)
    for i, (b0, b1, b2, a1, a2) in enumerate(sec):
        gin = np.prod([sec[l][0] for l in range(i)]) if i else 1.0
        b[2 * i:2 * i + 2] = np.array([b1 - a1 * b0, b2 - a2 * b0]) * gin
        c[2 * i] = np.prod([sec[l][0] for l in range(i + 1, S)]) if i + 1 < S else 1.0
    return b, c, float(np.prod([r[0] for r in sec]))


def model_matrix_cascade(x, sec, LC=32, NCH=96, SEG=12, state_in=None):
    """The matrix-core decomposition over one channel, in FP64: chunks of LC
    samples (y0 = Tc x, u = H x), chunk states in segments of SEG chunks from a
    zero state, the tile aggregate from the segment aggregates, the tile
    entering state P_{t+1} = Phi_T P_t + E_t, the segments' entering states,
    the chunks' entering states S, then y = y0 + G S."""
    F = _cascade_transition(sec)
    b, c, d = _cascade_io(sec)
    D = F.shape[0]
    h = np.zeros(LC)
    h[0] = d
    for n in range(1, LC):
        h[n] = c @ np.linalg.matrix_power(F, n - 1) @ b
    Tc = np.array([[h[r - m] if r >= m else 0.0 for m in range(LC)] for r in range(LC)])
    H = np.stack([np.linalg.matrix_power(F, LC - 1 - m) @ b for m in range(LC)], axis=1)
    G = np.stack([c @ np.linalg.matrix_power(F, r) for r in range(LC)])
    Fc = np.linalg.matrix_power(F, LC)
    Fs = np.linalg.matrix_power(Fc, SEG)
    PhiT = np.linalg.matrix_power(Fc, NCH)
    T = LC * NCH
    N = x.size
    nt = -(-N // T)
    xp = np.concatenate([x, np.zeros(nt * T - N)])
    y = np.empty_like(xp)
    P = np.zeros(D) if state_in is None else np.asarray(state_in, float).reshape(-1)
    for t in range(nt):
        X = xp[t * T:(t + 1) * T].reshape(NCH, LC).T
        Y0, U = Tc @ X, H @ X
        nseg = NCH // SEG
        g = np.zeros((nseg, D))
        for j in range(nseg):
            s = np.zeros(D)
            for m in range(SEG):
                s = Fc @ s + U[:, j * SEG + m]
            g[j] = s
        E = np.zeros(D)
        for j in range(nseg):
            E = Fs @ E + g[j]
        e = P.copy()
        Sx = np.zeros((D, NCH))
        for j in range(nseg):
            s = e.copy()
            for m in range(SEG):
                Sx[:, j * SEG + m] = s
                s = Fc @ s + U[:, j * SEG + m]
            e = Fs @ e + g[j]
        y[t * T:(t + 1) * T] = (Y0 + G @ Sx).T.reshape(-1)
        P = PhiT @ P + E
    return y[:N]


@pytest.mark.parametrize("S,N", [(1, 5000), (2, 3072), (4, 3 * 3072 + 77), (6, 2 * 3072 + 1), (8, 4000)])
def test_matrix_cascade_model_matches_oracle(S, N):
    from paper_2504_08624_amd import design, signals
    sec = design.random_sections(signals.rng(75, S), S, 0.5, 0.995)
    x = signals.rng(76, S).standard_normal(N)
    si = signals.rng(77, S).standard_normal((S, 2))
    y = model_matrix_cascade(x, sec, state_in=si)
    ref = O.sos(x[None], sec, state_in=si[None])[0]
    assert np.max(np.abs(y - ref)) < 1e-9 * max(1.0, np.max(np.abs(ref)))


def test_matrix_cascade_model_small_chunks():
    # the algebra does not depend on the sizes: chunks of 4, segments of 3,
    # 6 chunks a tile, many tiles
    from paper_2504_08624_amd import design, signals
    sec = design.random_sections(signals.rng(78), 3, 0.5, 0.99)
    x = signals.rng(79).standard_normal(24 * 9 + 5)
    y = model_matrix_cascade(x, sec, LC=4, NCH=6, SEG=3)
    ref = O.sos(x[None], sec)[0]
    assert np.max(np.abs(y - ref)) < 1e-10 * max(1.0, np.max(np.abs(ref)))
