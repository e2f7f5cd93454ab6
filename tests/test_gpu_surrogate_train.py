"""Surrogate training on the GPU against the oracle: the AdamW step (with
weight decay, decoupled from the gradient; biases undecayed), the reduced
basis (Eckart-Young optimality and the leading vectors with their sign
convention against numpy's SVD of the same targets), the ridge mismatch head
against least squares, and checkpoint/resume of the optimiser state."""

import sys

import numpy as np
import pytest

import oracle
from oracle import surrogate as OS
from paper_2407_19048_amd import gwgen, inputs
from paper_2407_19048_amd import surrogate as GS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gen():
    return gwgen.Generator(inputs.config("surrogate"))


def _bounds():
    cfg = inputs.config("surrogate")
    lo = np.array([cfg["mc"][0], cfg["q"][0], cfg["chi"][0], cfg["chi"][0]])
    hi = np.array([cfg["mc"][1], cfg["q"][1], cfg["chi"][1], cfg["chi"][1]])
    return lo, hi


def _batch(B, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = _bounds()
    theta = rng.uniform(lo, hi, (B, 4)).astype(np.float32)
    z = rng.standard_normal((B, 128)).astype(np.float32)
    return theta, z


def _flat_weights(seed):
    flat = GS.init_weights(seed, scale=1.0)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    flat = flat + (0.05 * rng.standard_normal(flat.shape)).astype(np.float32)
    flat[:16 * 256].reshape(16, 256)[4:] = 0.0
    return flat


def _split(flat):
    """[(W, b)] float64 in the oracle's shapes (layer 0 without the padding rows)."""
    out, o = [], 0
    for l, (nin, nout) in enumerate(GS.LAYERS):
        W = flat[o:o + nin * nout].reshape(nin, nout).astype(np.float64)
        o += nin * nout
        b = flat[o:o + nout].astype(np.float64)
        o += nout
        out.append([W[:4] if l == 0 else W, b])
    return out


def _oracle_adamw(flat, batches, lrs, wd, eps):
    """The oracle's training steps: bf16-emulating forward/backward, then
    AdamW on every weight (decayed) and bias (not decayed)."""
    lo, hi = _bounds()
    P = _split(flat)
    M = [[np.zeros_like(W), np.zeros_like(b)] for W, b in P]
    V = [[np.zeros_like(W), np.zeros_like(b)] for W, b in P]
    for t, ((theta, z), lr) in enumerate(zip(batches, lrs), start=1):
        x = OS.normalise_inputs(theta.astype(np.float64), lo, hi)
        out, cache = OS.mlp_forward([tuple(pw) for pw in P], x, emulate_bf16=True)
        _, dout = OS.mse_loss_and_grad(out, z.astype(np.float64))
        grads = OS.mlp_backward([tuple(pw) for pw in P], cache, dout, emulate_bf16=True)
        for l in range(len(P)):
            for j, decay in ((0, wd), (1, 0.0)):
                P[l][j], M[l][j], V[l][j] = OS.adamw_step(P[l][j], grads[l][j], M[l][j], V[l][j], t, lr, decay,
                                                         eps=eps)
    return P


def _gpu_steps(s, batches, lrs, wd):
    for (theta, z), lr in zip(batches, lrs):
        s.train_step(torch.from_numpy(theta).to(DEV), torch.from_numpy(z).to(DEV), lr, wd)
    torch.cuda.synchronize()
    return s.get_weights()


def test_train_step_matches_oracle_adamw(gen):
    """Three AdamW steps at a non-zero weight decay.  eps = 1 keeps the update
    smooth in the gradient (m_hat/(sqrt(v_hat) + 1)), so the comparison is
    limited only by the gradients' rounding differences: every tensor's
    displacement within 1e-3 relative L2 of the oracle's."""
    B = 256
    s = GS.Surrogate(gen, max_batch=B)
    flat = _flat_weights(41)
    s.set_weights(flat)
    s.set_adam(0.9, 0.999, 1.0)
    batches = [_batch(B, 50 + t) for t in range(3)]
    lrs = [3e-2, 2e-2, 1e-2]
    wd = 0.5
    got = _split(_gpu_steps(s, batches, lrs, wd))
    ref = _oracle_adamw(flat, batches, lrs, wd, 1.0)
    p0 = _split(flat)
    rels = []
    for l in range(len(p0)):
        for j in (0, 1):
            d_gpu = got[l][j] - p0[l][j]
            d_orc = ref[l][j] - p0[l][j]
            rels.append(np.linalg.norm(d_gpu - d_orc) / np.linalg.norm(d_orc))
    _say("AdamW (eps 1, wd %.1f) displacement rel L2 per tensor: %s" % (wd, " ".join("%.1e" % r for r in rels)))
    assert max(rels) < 1e-3


def test_train_step_default_eps_first_step(gen):
    """One step with the default eps = 1e-8: each weight moves by
    lr (sign(g) + wd p) up to eps.  Checked element by element wherever the
    oracle's gradient is clear of zero (|g| above 1e-2 of the tensor's RMS
    and above 1e4 eps, where the bfloat16 gradients of the two sides cannot
    disagree in sign and eps does not amplify their rounding); over all
    elements at most 2 % may differ (all of them with |g| near 0)."""
    B = 256
    s = GS.Surrogate(gen, max_batch=B)
    flat = _flat_weights(43)
    s.set_weights(flat)
    batch = _batch(B, 60)
    lr, wd = 1e-3, 0.1
    got = _split(_gpu_steps(s, [batch], [lr], wd))
    ref = _oracle_adamw(flat, [batch], [lr], wd, 1e-8)
    lo, hi = _bounds()
    P = [tuple(pw) for pw in _split(flat)]
    x = OS.normalise_inputs(batch[0].astype(np.float64), lo, hi)
    out, cache = OS.mlp_forward(P, x, emulate_bf16=True)
    _, dout = OS.mse_loss_and_grad(out, batch[1].astype(np.float64))
    grads = OS.mlp_backward(P, cache, dout, emulate_bf16=True)
    checked = total = differ = 0
    for l in range(len(P)):
        for j in (0, 1):
            g = grads[l][j]
            # clear of zero relative to the tensor and to eps (near |g| ~ eps
            # the step g/(|g| + eps) amplifies gradient rounding)
            ok = np.abs(g) > max(1e-2 * np.sqrt(np.mean(g * g)), 1e4 * 1e-8)
            # up to 1e-5 of the step plus the binary32 rounding of the weight
            tol = 1e-5 * lr + 2.4e-7 * np.abs(ref[l][j])
            off = np.abs(got[l][j] - ref[l][j]) > tol
            assert not (off & ok).any(), (l, j, int((off & ok).sum()))
            checked += int(ok.sum())
            total += g.size
            differ += int(off.sum())
    _say("AdamW default eps: %d of %d elements checked one by one; %d differ (gradient near 0)"
         % (checked, total, differ))
    assert differ <= 0.02 * total
    assert checked >= 0.5 * total


def test_weight_decay_is_decoupled_on_gpu(gen):
    """Targets equal to the network's own output give exactly zero
    gradients: the moments stay zero and the step is pure decay,
    W <- W (1 - lr wd), with the biases unchanged."""
    B = 128
    s = GS.Surrogate(gen, max_batch=B)
    flat = _flat_weights(45)
    s.set_weights(flat)
    theta, _ = _batch(B, 61)
    th = torch.from_numpy(theta).to(DEV)
    out = torch.empty((B, 128), dtype=torch.float32, device=DEV)
    s.forward(th, out)
    lr, wd = 1e-2, 0.25
    s.train_step(th, out.clone(), lr, wd)
    torch.cuda.synchronize()
    got, p0 = _split(s.get_weights()), _split(flat)
    for l in range(len(p0)):
        np.testing.assert_allclose(got[l][0], p0[l][0] * (1 - lr * wd), rtol=3e-7, atol=1e-30)
        np.testing.assert_array_equal(got[l][1], p0[l][1])


def test_checkpoint_resume_is_bit_identical(gen, tmp_path):
    """Training interrupted by save/load continues exactly as without the
    interruption (weights, AdamW moments, step counter and hyper-parameters
    are in the file); a file without the optimiser state (the earlier
    format) loads with fresh moments."""
    B = 256
    batches = [_batch(B, 70 + t) for t in range(5)]
    lrs = [1e-3] * 5
    a = GS.Surrogate(gen, max_batch=B)
    a.set_weights(_flat_weights(47))
    a.set_adam(0.85, 0.99, 1e-7)
    _gpu_steps(a, batches[:3], lrs[:3], 0.01)
    path = str(tmp_path / "ckpt.bin")
    a.save(path)
    wa = _gpu_steps(a, batches[3:], lrs[3:], 0.01)
    b = GS.Surrogate(gen, max_batch=B)
    b.load(path)
    wb = _gpu_steps(b, batches[3:], lrs[3:], 0.01)
    assert np.array_equal(wa, wb)
    # the earlier format: header "GWSURR1", state and weights, no optimiser state
    raw = open(path, "rb").read()
    n_state = 4 * 2 * 64 * 1024 + 8 * 2 * 1024 + 4 * 9 * 128 + 4 * 128 * 2 + 4 * 257
    n_w = 4 * a.n_weights
    v1 = str(tmp_path / "v1.bin")
    with open(v1, "wb") as fh:
        fh.write(b"GWSURR1\x00" + raw[8:8 + n_state + n_w])
    c = GS.Surrogate(gen, max_batch=B)
    c.load(v1)
    d = GS.Surrogate(gen, max_batch=B)
    d.load(path)
    d.set_weights(d.get_weights())  # same weights, fresh moments, step 0
    d.set_adam(0.9, 0.999, 1e-8)    # the defaults a file without them loads with
    assert np.array_equal(_gpu_steps(c, batches[:1], lrs[:1], 0.01), _gpu_steps(d, batches[:1], lrs[:1], 0.01))
    with pytest.raises(gwgen.GWError):
        GS.Surrogate(gen, max_batch=B).load(str(tmp_path / "missing.bin"))
    trunc = str(tmp_path / "trunc.bin")
    with open(trunc, "wb") as fh:
        fh.write(raw[:len(raw) - 9])
    with pytest.raises(gwgen.GWError):
        GS.Surrogate(gen, max_batch=B).load(trunc)


def _oracle_targets(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = _bounds()
    th = rng.uniform(lo, hi, (n, 4))
    R = np.empty((n, 1024))
    D = np.empty((n, 1024))
    for i in range(n):
        R[i], D[i] = OS.targets(*th[i])
    return R, D


def test_reduced_basis_matches_oracle(gen):
    """Basis of 20480 target sets of the oracle (uploaded as binary32):
    the mean to binary64 rounding, orthonormal vectors, a truncation error
    equal to the optimum (the discarded squared singular values of numpy's
    SVD) to 1e-6 of the total energy, and the leading vectors (well
    separated singular values) equal to the oracle's with its sign
    convention."""
    n = 20480
    R, D = _oracle_targets(n, 81)
    R32, D32 = R.astype(np.float32), D.astype(np.float32)
    s = GS.Surrogate(gen, max_batch=256)
    s.fit_basis(torch.from_numpy(R32).to(DEV), torch.from_numpy(D32).to(DEV))
    basis, mean, _, _, _, _ = s.get_state()
    for part, X in enumerate((R32.astype(np.float64), D32.astype(np.float64))):
        m_o, V_o = OS.reduced_basis(X, 64)
        np.testing.assert_allclose(mean[part], m_o, rtol=1e-12, atol=1e-12 * np.abs(m_o).max())
        V = basis[part].astype(np.float64)
        np.testing.assert_allclose(V @ V.T, np.eye(64), atol=2e-6)
        total = float(np.sum((X - m_o) ** 2))
        sv = np.linalg.svd(X - m_o, compute_uv=False)
        opt = float(np.sum(sv[64:] ** 2))
        err = OS.truncation_error(X, m_o, V)
        _say("basis part %d: truncation %.6e (optimum %.6e, total %.3e)" % (part, err, opt, total))
        assert abs(err - opt) <= 1e-6 * total
        # vectors whose squared singular value is separated from both
        # neighbours by more than 1e-8 of the largest (the binary64 Gram
        # matrices of the two sides differ by rounding far below that)
        gaps = (sv[:15] ** 2 - sv[1:16] ** 2) / sv[0] ** 2
        lead = [k for k in range(15) if gaps[k] > 1e-8 and (k == 0 or gaps[k - 1] > 1e-8)]
        _say("basis part %d: %d leading vectors compared" % (part, len(lead)))
        assert len(lead) >= 4
        for k in lead:
            np.testing.assert_allclose(V[k], V_o[k], atol=1e-4)


def test_ridge_head_matches_least_squares(gen):
    n = 2048
    rng = np.random.Generator(np.random.PCG64(91))
    h3 = rng.standard_normal((n, 256)).astype(np.float32)
    mm = 10 ** rng.uniform(-6, -1, n)
    mm[:3] = (0.0, -1e-16, 1e-13)   # below the floor: log10 of 1e-12
    s = GS.Surrogate(gen, max_batch=256)
    s.fit_head(torch.from_numpy(h3).to(DEV), mm, 1e-4)
    head = s.get_state()[5].astype(np.float64)
    ref = OS.ridge_head(h3.astype(np.float64), np.log10(np.maximum(mm, 1e-12)), 1e-4)
    rel = np.linalg.norm(head - ref) / np.linalg.norm(ref)
    _say("ridge head rel L2 %.2e" % rel)
    assert rel < 1e-5
    with pytest.raises(gwgen.GWError):
        s.fit_head(torch.from_numpy(h3).to(DEV), np.full(n, np.nan), 1e-4)
