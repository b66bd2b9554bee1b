"""GPU parity and training of the candidate-vetting network (forward, gradients, Adam, fused capture)."""
import numpy as np
import pytest
import torch as _torch  # imported at collection: the first import on a fresh box is slow

import synth
from oracle import fstat_oracle as ora
from oracle import vet_data
from oracle import vet_oracle as vo
from tests.gpu_util import dev, make_plan, note

pytestmark = pytest.mark.gpu

BF16_LAYERS = ("w2", "w3", "w4", "w5")   # weights used as BF16 matrix-core operands


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _theta(seed=3):
    rng = np.random.default_rng(seed)
    th = vo.init_params(rng)
    th += 0.02 * rng.standard_normal(th.size) * (np.arange(th.size) >= 0)
    return th.astype(np.float32).astype(np.float64)


def _as_gpu_weights(theta):
    """The FP32 master vector with the matrix-product weights rounded to BF16, as the GPU uses them."""
    p = vo.unflatten(theta.copy())
    for k in BF16_LAYERS:
        p[k] = vo.bf16_round(p[k]).reshape(p[k].shape)
    return vo.flatten(p)


def _patches(rng, n):
    scale = rng.uniform(1.0, 6.0, size=(n, 1))
    return (rng.chisquare(4, size=(n, 256)) * scale).astype(np.float32)


def test_forward_matches_fp64_reference(torch):
    from paper_1410_3677_amd import fstat as F
    rng = np.random.default_rng(11)
    theta = _theta()
    v = F.Vetter(64)
    v.set_params(theta.astype(np.float32))
    x = _patches(rng, 150)   # more than one batch
    logits = torch.empty(150, device="cuda")
    v.forward(torch.as_tensor(x, device="cuda"), logits)
    got = logits.cpu().numpy().astype(np.float64)
    ref = vo.forward(_as_gpu_weights(theta), x.astype(np.float64))
    err = np.abs(got - ref)
    note(f"logit err max {err.max():.3e}, logit scale {np.abs(ref).max():.3f}")
    # BF16 activations (relative rounding 2^-9 per layer, four layers): bound 2% of the scale
    assert err.max() <= 0.02 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("n,batch", [(1, 8192), (3, 8192), (17, 8)])
def test_forward_of_few_patches(torch, n, batch):
    # fewer items than one workgroup's wavefronts (a grid of one workgroup), and a batch
    # size that ends a batch inside a workgroup's share of items
    from paper_1410_3677_amd import fstat as F
    rng = np.random.default_rng(100 + n)
    theta = _theta(7)
    v = F.Vetter(batch)
    v.set_params(theta.astype(np.float32))
    x = _patches(rng, n)
    x[0, :5] = 0.0                       # zero 2F at the left edge of the first patch
    logits = torch.full((n + 1,), 7.5, device="cuda")
    v.forward(torch.as_tensor(x, device="cuda"), logits[:n])
    got = logits.cpu().numpy().astype(np.float64)
    assert got[n] == 7.5                 # nothing written past the last patch
    ref = vo.forward(_as_gpu_weights(theta), x.astype(np.float64))
    err = np.abs(got[:n] - ref)
    note(f"{n} patches, batch {batch}: logit err max {err.max():.3e}, scale {np.abs(ref).max():.3f}")
    assert err.max() <= 0.02 * max(1.0, np.abs(ref).max())


def test_gradients_match_fp64_reference(torch):
    from paper_1410_3677_amd import fstat as F
    rng = np.random.default_rng(12)
    theta = _theta(4)
    v = F.Vetter(64)
    v.set_params(theta.astype(np.float32))
    x = _patches(rng, 64)
    y = (rng.uniform(size=64) < 0.5).astype(np.float32)
    g = torch.empty(vo.N_PARAMS, device="cuda")
    loss = torch.empty(1, device="cuda")
    v.gradient(torch.as_tensor(x, device="cuda"), torch.as_tensor(y, device="cuda"), loss, g)
    torch.cuda.synchronize()
    ref_loss, ref_g = vo.loss_and_grad(_as_gpu_weights(theta), x.astype(np.float64), y.astype(np.float64))
    gg = vo.unflatten(g.cpu().numpy().astype(np.float64))
    rg = vo.unflatten(ref_g)
    assert abs(float(loss.item()) - ref_loss) < 1e-2 * max(1.0, ref_loss)
    for name, _ in vo.SHAPES:
        a, b = gg[name].ravel(), rg[name].ravel()
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-30))
        rel = float(np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-30))
        note(f"{name}: cosine {cos:.6f} rel-L2 {rel:.2e}")
        assert cos >= 0.999 and rel <= 2e-2, name


def _train(F, torch, x, y, epochs, seed, batch=256, lr=1e-3):
    v = F.Vetter(batch)
    v.set_params(vo.init_params(np.random.default_rng(seed)).astype(np.float32))
    xg, yg = torch.as_tensor(x, device="cuda"), torch.as_tensor(y, device="cuda")
    rng = np.random.default_rng(seed + 1)
    loss = torch.empty(1, device="cuda")
    hist = []
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(len(y)), device="cuda")
        for i in range(0, len(y) - batch + 1, batch):
            idx = perm[i:i + batch]
            v.gradient(xg[idx].contiguous(), yg[idx].contiguous(), loss)
            v.adam_step(lr)
        hist.append(float(loss.item()))
    return v, hist


def operating_point(logit_inj, logit_noise, max_added_dismissal=0.01):
    """Cut that keeps all but max_added_dismissal of the injections; fraction of noise kept."""
    cut = np.quantile(logit_inj, max_added_dismissal)
    return float(cut), float(np.mean(logit_noise >= cut)), float(np.mean(logit_inj < cut))


def test_training_on_oracle_patches_beats_the_threshold_alone(torch):
    from paper_1410_3677_amd import fstat as F
    note("generating oracle patches")
    x, y, st = vet_data.make_dataset(5000, 16, 600, 8)
    xe, ye, ste = vet_data.make_dataset(5001, 6, 400, 6)
    note(f"train {len(y)} eval {len(ye)}; threshold false dismissal {st['threshold_false_dismissal']:.4f}")
    v, hist = _train(F, torch, x, y, epochs=4, seed=21)
    note(f"loss by epoch {hist}")
    assert hist[-1] < 0.2
    le = torch.empty(len(ye), device="cuda")
    v.forward(torch.as_tensor(xe, device="cuda"), le)
    le = le.cpu().numpy()
    cut, far, fdr = operating_point(le[ye == 1], le[ye == 0])
    note(f"held out: at <= 1% added false dismissal the network keeps {far:.4f} of the noise crossings "
         f"(the threshold alone keeps all of them)")
    assert fdr <= 0.011
    assert far < 0.5


@pytest.mark.parametrize("precision,ib", [(1, 0), (1, 1), (0, 0), (0, 1)])
def test_fused_capture_scores_equal_network_on_search_spectra(torch, precision, ib):
    from paper_1410_3677_amd import fstat as F
    note(f"fused patch capture after the F kernel, precision={precision}, interbinning={ib}")
    w = synth.workload("full")
    seg = w.segments[0]
    nfft = synth.nfft_for(seg.n)
    nb = nfft // 2
    al, de, fd = w.alpha[:2], w.delta[:2], w.fdot[:3]
    v = F.Vetter(512)
    v.set_params(_theta(5).astype(np.float32))
    plan = make_plan([seg], use_graph=0, interbinning=ib, precision=precision)
    plan.attach_vetter(v, 1 << 16)
    plan.search_batch(0, dev(al), dev(de), dev(fd))
    plan.vet_candidates()
    recs, keys, n = plan.candidates()
    assert n > 100 and np.all(np.isfinite(keys["vet_score"]))
    # the same network on windows of the 2F spectrum of the same templates
    spec = torch.empty(len(al) * len(fd) * nb, dtype=torch.float64 if precision == 0 else torch.float32,
                       device="cuda")
    plain = make_plan([seg], use_graph=0, interbinning=ib, precision=precision)
    plain.twoF_spectrum(0, dev(al), dev(de), dev(fd), spec)
    s = spec.view(len(al), len(fd), nb).cpu().numpy().astype(np.float32)   # the capture's FP32 rows
    win = np.zeros((n, 256), np.float32)
    for i, (a, f, b) in enumerate(zip(keys["sky"], keys["fdot_idx"], keys["bin"])):
        lo, hi = b - 128, b + 128
        src = s[a, f, max(lo, 0):min(hi, nb)]
        win[i, max(lo, 0) - lo:max(lo, 0) - lo + src.size] = src
    lg = torch.empty(n, device="cuda")
    v.forward(torch.as_tensor(win, device="cuda"), lg)
    ref = 1.0 / (1.0 + np.exp(-lg.cpu().numpy()))
    # The search kernel and the spectrum kernel are separate instantiations whose FFT
    # arithmetic the compiler may contract differently (last-bit differences in 2F); such a
    # difference can flip one BF16 rounding inside the network (2^-9 relative).
    diff = np.abs(keys["vet_score"] - ref)
    note(f"scores: {np.mean(diff == 0):.3f} bitwise equal, max difference {diff.max():.2e}")
    assert diff.max() < 2e-3
    assert np.mean(diff == 0) > 0.5


def test_fused_capture_on_a_bin_range(torch):
    # a bin range other than [0, nfft/2), here across nfft/2: the capturing second pass
    # stores all P outputs of its rows, and the capture reads bins outside the range as 0.
    # On this range the search's and the spectrum kernel's 2F differ in the last bit on
    # about a sixth of the bins (instantiations contracted differently), so more BF16
    # roundings in the network flip than on the default range.
    from paper_1410_3677_amd import fstat as F
    w = synth.workload("full")
    seg = w.segments[0]
    k0, k1 = 70000, 140000
    al, de, fd = w.alpha[:2], w.delta[:2], w.fdot[:3]
    v = F.Vetter(512)
    v.set_params(_theta(5).astype(np.float32))
    plan = make_plan([seg], use_graph=0, precision=1, k_min=k0, k_max=k1)
    plan.attach_vetter(v, 1 << 16)
    plan.search_batch(0, dev(al), dev(de), dev(fd))
    plan.vet_candidates()
    recs, keys, n = plan.candidates()
    note(f"bins [{k0}, {k1}): {n} crossings")
    assert n > 100 and np.all(np.isfinite(keys["vet_score"]))
    assert keys["bin"].min() >= k0 and keys["bin"].max() < k1
    nb = k1 - k0
    spec = torch.empty(len(al) * len(fd) * nb, dtype=torch.float32, device="cuda")
    plain = make_plan([seg], use_graph=0, precision=1, k_min=k0, k_max=k1)
    plain.twoF_spectrum(0, dev(al), dev(de), dev(fd), spec)
    s = spec.view(len(al), len(fd), nb).cpu().numpy()
    win = np.zeros((n, 256), np.float32)
    for i, (a, f, b) in enumerate(zip(keys["sky"], keys["fdot_idx"], keys["bin"])):
        lo, hi = max(b - 128, k0), min(b + 128, k1)
        win[i, lo - (b - 128):hi - (b - 128)] = s[a, f, lo - k0:hi - k0]
    lg = torch.empty(n, device="cuda")
    v.forward(torch.as_tensor(win, device="cuda"), lg)
    ref = 1.0 / (1.0 + np.exp(-lg.cpu().numpy()))
    diff = np.abs(keys["vet_score"] - ref)
    note(f"scores: {np.mean(diff == 0):.3f} bitwise equal, max difference {diff.max():.2e}")
    assert diff.max() < 2e-3
    assert np.mean(diff == 0) > 0.5


def test_capture_in_a_plan_of_two_lengths_equals_a_plan_of_one(torch):
    """With the library's batch sizes, a plan's launches hold more templates for a segment
    whose transform is shorter than the plan's longest (the same intermediate memory and
    launch-sized 2F rows): here one launch of 512 templates instead of two of 256.  That
    segment's candidates, 2F and captured-patch scores equal those of a plan of the
    segment alone."""
    from paper_1410_3677_amd import fstat as F
    w = synth.workload("full")
    long_seg = w.segments[0]
    rng = np.random.default_rng(31)
    injs = synth.draw_injections(rng, 1, 15.0, 15.0)
    short = synth.make_segment(30000, 2.0, 100.0, 1.0, 7031, injs)
    assert 4 * synth.nfft_for(short.n) == synth.nfft_for(long_seg.n)
    al, de, fd = w.alpha[:8], w.delta[:8], w.fdot[:64]
    v = F.Vetter(512)
    v.set_params(_theta(5).astype(np.float32))
    found = []
    for segs, s in (([long_seg, short], 1), ([short], 0)):
        plan = make_plan(segs, use_graph=0, precision=1)   # the library's batch sizes
        plan.attach_vetter(v, 1 << 16)
        plan.search_batch(s, dev(al), dev(de), dev(fd))
        plan.vet_candidates()
        found.append(plan.candidates())
    (r0, k0, n0), (r1, k1, n1) = found
    note(f"short segment in a plan of two lengths: {n0} crossings, alone: {n1}")
    assert n0 == n1 and n0 > 100
    for f in ("sky", "fdot_idx", "bin"):
        np.testing.assert_array_equal(k0[f], k1[f])
    np.testing.assert_array_equal(r0["twoF"], r1["twoF"])
    assert np.all(np.isfinite(k0["vet_score"]))
    np.testing.assert_array_equal(k0["vet_score"], k1["vet_score"])
