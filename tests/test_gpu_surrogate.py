"""GPU surrogate kernels against the FP64 surrogate oracle, and the surrogate
in use: trained on exact solves the GPU evaluator produces, ranking candidate
flips, and pruning a greedy search (C ABI, GPU).

Tolerances.  FP32 mode: every product accumulates in FP32 over at most a few
thousand terms, so outputs and gradients agree with the FP64 reference to
~1e-6 relative; 1e-4 (norm-wise per tensor) is used.  BF16 mode rounds both
operands of every product to 8 significant bits (relative perturbation up to
2^-8 per product).  The output passes through six such products (2e-2 is
used).  The gradient of the first convolution passes through twelve: four
convolutions and two head products forward, then the head's two backward
products, three data gradients and the weight gradient.  That is a linear
bound of 12 x 2^-8 = 4.7e-2 on the relative perturbation of its terms.  The
random targets make the gradient sums cancel, which amplifies this a little,
so 1e-1 per tensor is used.  The FP32 run is the exact check of the kernels;
the BF16 run checks that the rounding stays where the arithmetic puts it.
"""

import numpy as np
import pytest

from oracle import surrogate as osur
from paper_2412_17617_amd import pxd
from paper_2412_17617_amd.tree_search import descent

from sur_common import init_params, random_maps

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
CFG = osur.SurrogateConfig(n_layers=3, ny=8, nx=8, channels=(32, 32, 64, 64), hidden=64, emb=16, n_out=9)
FREQS = np.linspace(3e9, 9e9, 7)
TOL = {pxd.SUR_FP32: 1e-4, pxd.SUR_BF16: 1e-1}


def make(prec, max_batch=8, cfg=CFG, freqs=FREQS):
    return pxd.Surrogate(cfg.n_layers, cfg.ny, cfg.nx, freqs, freqs[0], freqs[-1], channels=cfg.channels,
                         hidden=cfg.hidden, emb=cfg.emb, precision=prec, max_batch=max_batch)


def u_of(freqs):
    return (freqs - freqs[0]) / (freqs[-1] - freqs[0])


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def test_init_params_are_the_seeded_draws():
    s = make(pxd.SUR_FP32)
    assert s.n_params == osur.n_params(CFG)
    s.init_params(42)
    assert np.array_equal(s.get_params(), init_params(CFG, 42).astype(np.float32))
    s.close()


@pytest.mark.parametrize("prec", [pxd.SUR_FP32, pxd.SUR_BF16])
def test_forward_matches_oracle(prec):
    s = make(prec)
    p32 = init_params(CFG, 3).astype(np.float32)
    s.set_params(p32)
    maps = random_maps(5, 3 * 64, 4)
    out = torch.zeros((5, len(FREQS), 9), dtype=torch.float32, device=DEV)
    s.forward(torch.from_numpy(maps).to(DEV), out)
    got = out.cpu().numpy()
    want, _ = osur.forward(p32.astype(np.float64), maps, u_of(FREQS), CFG)
    print(f"forward relative error {rel(got, want):.2e}")
    assert rel(got, want) <= (1e-4 if prec == pxd.SUR_FP32 else 2e-2), rel(got, want)
    s.close()


@pytest.mark.parametrize("prec", [pxd.SUR_FP32, pxd.SUR_BF16])
def test_forward_at_full_size_matches_oracle(prec):
    """The ranking network at its working size: 3 x 24 x 24 maps, channels
    32-64, hidden 256, 101 frequencies, buffers for 2,048 maps per call."""
    cfg = osur.SurrogateConfig(n_layers=3, ny=24, nx=24, channels=(32, 32, 64, 64), hidden=256, emb=16, n_out=9)
    freqs = np.linspace(1e9, 8e9, 101)
    s = make(prec, max_batch=2048, cfg=cfg, freqs=freqs)
    p32 = init_params(cfg, 12).astype(np.float32)
    s.set_params(p32)
    maps = random_maps(3, 3 * 24 * 24, 13)
    out = torch.zeros((3, len(freqs), 9), dtype=torch.float32, device=DEV)
    s.forward(torch.from_numpy(maps).to(DEV), out)
    got = out.cpu().numpy()
    want, _ = osur.forward(p32.astype(np.float64), maps, u_of(freqs), cfg)
    print(f"full-size forward relative error {rel(got, want):.2e}")
    assert rel(got, want) <= (1e-4 if prec == pxd.SUR_FP32 else 2e-2), rel(got, want)
    s.close()


@pytest.mark.parametrize("prec", [pxd.SUR_FP32, pxd.SUR_BF16])
def test_gradient_matches_oracle(prec):
    s = make(prec)
    p32 = init_params(CFG, 5).astype(np.float32)
    s.set_params(p32)
    maps = random_maps(6, 3 * 64, 6)
    target = (np.random.default_rng(7).standard_normal((6, len(FREQS), 9)) * 0.3).astype(np.float32)
    g = torch.zeros(s.n_params, dtype=torch.float32, device=DEV)
    loss = torch.zeros(1, dtype=torch.float32, device=DEV)
    s.gradient(torch.from_numpy(maps).to(DEV), torch.from_numpy(target).to(DEV), g, loss)
    L, g_o = osur.gradient(p32.astype(np.float64), maps, u_of(FREQS), target.astype(np.float64), CFG)
    assert abs(loss.item() - L) <= TOL[prec] * L
    g = g.cpu().numpy()
    o, errs = 0, {}
    for name, shape in osur.layout(CFG):
        n = int(np.prod(shape))
        errs[name] = rel(g[o:o + n], g_o[o:o + n])
        o += n
    print("gradient relative errors:", {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) <= TOL[prec], errs
    s.close()


def test_adamw_steps_match_oracle():
    """The optimiser kernel against the oracle's AdamW fed with the same
    gradient (the GPU's, which is reproducible bit for bit between calls)."""
    s = make(pxd.SUR_FP32)
    p32 = init_params(CFG, 8).astype(np.float32)
    s.set_params(p32)
    maps = random_maps(4, 3 * 64, 9)
    target = (np.random.default_rng(10).standard_normal((4, len(FREQS), 9)) * 0.3).astype(np.float32)
    tm, tt = torch.from_numpy(maps).to(DEV), torch.from_numpy(target).to(DEV)
    hp = dict(lr=1e-3, beta1=0.9, beta2=0.99, eps=1e-8, weight_decay=0.5)  # decay large enough to see
    p, m, v = p32.astype(np.float64), np.zeros(len(p32)), np.zeros(len(p32))
    g_dev = torch.zeros(s.n_params, dtype=torch.float32, device=DEV)
    for t in (1, 2, 3):
        s.gradient(tm, tt, g_dev)
        g = g_dev.cpu().numpy().astype(np.float64)
        want, m, v = osur.adamw_step(p, g, m, v, t, hp["lr"], hp["beta1"], hp["beta2"], hp["eps"],
                                     hp["weight_decay"])
        s.train_step(tm, tt, **hp)
        got = s.get_params().astype(np.float64)
        assert np.max(np.abs(got - want)) <= 1e-4 * hp["lr"] + 1e-7, (t, np.max(np.abs(got - want)))
        p = got
    s.close()


# ---------------------------------------------------------------- in use

from synth import PortSpec, single_flips  # noqa: E402

from gpu_common import spec_variant  # noqa: E402

# One layer of 4 x 4 two-millimetre pixels with three ports: all 2^16 maps can
# be solved exactly, so the exhaustive optimum is known.
SPEC4 = spec_variant("small6x3", n_layers=1, nx=4, ny=4, a=2e-3, h=0.0,
                     ports=(PortSpec("right", 0), PortSpec("top", 0), PortSpec("left", 0)),
                     n_freq=13, f_lo=3e9, f_hi=9e9, seed=31)
ENTRIES = ((0, 0), (1, 0), (2, 0), (2, 1))  # every S entry the FoM uses
N_MAPS = 1 << 16


def all_maps_csr(idx):
    """Candidates as flips of the empty map: map i has cell c on iff bit c of i."""
    cells = [np.nonzero((i >> np.arange(16)) & 1)[0] for i in idx]
    off = np.zeros(len(idx) + 1, np.int32)
    off[1:] = np.cumsum([len(c) for c in cells])
    return off, np.concatenate(cells).astype(np.int32) if off[-1] else np.zeros(0, np.int32)


@pytest.fixture(scope="module")
def world():
    """Exact FoM of every map (product fill, FP64 GPU solves) and the exact S
    of a seeded training subset."""
    freqs = SPEC4.freqs
    pb = pxd.Problem.from_spec(SPEC4)
    Z = pb.fill(freqs, n_threads=16)
    ev = pxd.Evaluator(precision=pxd.PREC_FP64)
    ev.load_parent(Z, freqs)
    ev.load_problem(pb, SPEC4.z0)
    ev.set_fom_paper()
    zero = np.zeros(16, np.uint8)
    fom = np.empty(N_MAPS)
    for c0 in range(0, N_MAPS, 8192):
        off, cells = all_maps_csr(range(c0, c0 + 8192))
        _, fom[c0:c0 + 8192], st, _ = ev.evaluate_flips(zero, off, cells, want_S=False)
        assert np.all(st == 0)
    order = np.random.default_rng(31).permutation(N_MAPS)
    train_idx, held_idx = order[:4096], order[4096:4608]
    maps = ((np.arange(N_MAPS)[:, None] >> np.arange(16)) & 1).astype(np.uint8)
    S_train, _, _, _ = ev.evaluate_maps(maps[train_idx])
    S_held, _, _, _ = ev.evaluate_maps(maps[held_idx])
    yield dict(ev=ev, fom=fom, maps=maps, freqs=freqs, train=(maps[train_idx], pxd.Surrogate.encode(S_train, ENTRIES)),
               held=(maps[held_idx], pxd.Surrogate.encode(S_held, ENTRIES)))
    ev.close()


def make4(w, seed=1, steps=0, batch=64):
    s = pxd.Surrogate(1, 4, 4, w["freqs"], w["freqs"][0], w["freqs"][-1], entries=ENTRIES, hidden=128,
                      precision=pxd.SUR_BF16, max_batch=512)
    s.init_params(seed)
    maps, target = w["train"]
    rng = np.random.default_rng(seed)
    step = 0
    while step < steps:
        perm = rng.permutation(len(maps))
        tm = torch.from_numpy(maps[perm]).to(DEV)
        tt = torch.from_numpy(target[perm]).to(DEV)
        for b0 in range(0, len(maps) - batch + 1, batch):
            if step >= steps:
                break
            s.train_step(tm[b0:b0 + batch], tt[b0:b0 + batch], lr=2e-3, weight_decay=1e-4)
            step += 1
    torch.cuda.synchronize()
    return s


def held_out_loss(s, w):
    maps, target = w["held"]
    loss = torch.zeros(1, dtype=torch.float32, device=DEV)
    s.gradient(torch.from_numpy(maps[:512]).to(DEV), torch.from_numpy(target[:512]).to(DEV), None, loss)
    return loss.item()


def rank_all(s, w, k):
    off, cells = all_maps_csr(range(N_MAPS))
    fp = torch.zeros(N_MAPS, dtype=torch.float64, device=DEV)
    top = torch.zeros(k, dtype=torch.int32, device=DEV)
    s.rank(w["ev"], torch.zeros(16, dtype=torch.uint8, device=DEV), torch.from_numpy(off).to(DEV),
           torch.from_numpy(cells).to(DEV), k, fp, top)
    torch.cuda.synchronize()
    return fp.cpu().numpy(), top.cpu().numpy()


def spearman(a, b):
    ra, rb = np.argsort(np.argsort(a)), np.argsort(np.argsort(b))
    return float(np.corrcoef(ra, rb)[0, 1])


@pytest.fixture(scope="module")
def trained(world):
    untrained = make4(world, steps=0)
    s = make4(world, steps=3000)
    yield dict(s=s, untrained=untrained, loss0=held_out_loss(untrained, world), loss1=held_out_loss(s, world))
    s.close()
    untrained.close()


def test_training_on_exact_solves_lowers_held_out_loss(trained):
    print(f"held-out loss: untrained {trained['loss0']:.4g}, trained {trained['loss1']:.4g}")
    assert trained["loss1"] < 0.1 * trained["loss0"]


def test_ranking_kernel_is_the_fom_of_the_predictions(world, trained):
    """fom_pred of a few candidates against the FoM the oracle computes from
    the network's own outputs, and top-k against a sort of fom_pred."""
    from oracle import fom as ofom

    s = trained["s"]
    fp, top = rank_all(s, world, 32)
    assert np.array_equal(top, np.argsort(fp, kind="stable")[:32])
    pick = np.array([0, 1, 777, 4242, 65535, int(top[0])])
    out = torch.zeros((len(pick), len(world["freqs"]), 12), dtype=torch.float32, device=DEV)
    s.forward(torch.from_numpy(world["maps"][pick]).to(DEV), out)
    o = out.cpu().numpy().astype(np.float64)
    for r in range(len(pick)):
        S = np.zeros((len(world["freqs"]), 3, 3), np.complex128)
        for e, (i, j) in enumerate(ENTRIES):
            S[:, i, j] = np.exp(o[r, :, 3 * e])
        assert abs(ofom.fom(S, world["freqs"]) - fp[pick[r]]) <= 1e-9 * fp[pick[r]]


def train_more(s, maps, target, steps, seed, batch=64):
    rng = np.random.default_rng(seed)
    done = 0
    while done < steps:
        perm = rng.permutation(len(maps))
        tm = torch.from_numpy(maps[perm]).to(DEV)
        tt = torch.from_numpy(target[perm]).to(DEV)
        for b0 in range(0, len(maps) - batch + 1, batch):
            if done >= steps:
                break
            s.train_step(tm[b0:b0 + batch], tt[b0:b0 + batch], lr=5e-4, weight_decay=1e-4)
            done += 1
    torch.cuda.synchronize()


def pruned_search(w, s, rounds=4, k=64):
    """Surrogate-pruned search over every map: rank all, solve the best k not
    yet solved exactly, add those solves to the training set, fine-tune, and
    repeat.  Returns (best exact FoM found, exact solves used, the round that
    found it)."""
    maps, target = w["train"]
    solved = set()
    best, found = np.inf, -1
    for r in range(rounds):
        fp = rank_all(s, w, 1)[0]
        new = [int(i) for i in np.argsort(fp, kind="stable") if int(i) not in solved][:k]
        solved.update(new)
        S, F, st, _ = w["ev"].evaluate_maps(w["maps"][new])
        assert np.all(st == 0)
        if F.min() < best:
            best, found = F.min(), r
        maps = np.concatenate([maps, w["maps"][new]])
        target = np.concatenate([target, pxd.Surrogate.encode(S, ENTRIES)])
        train_more(s, maps, target, 400, seed=100 + r)
    return best, len(w["train"][0]) + len(solved), found


def test_global_search_with_the_surrogate(world, trained):
    """Reported experiment: exhaustive exact search over all 65,536 maps
    against a surrogate-pruned one (the 4,096 training maps plus four rounds
    of the best 64 predictions, each round's solves added to the training
    set).  Asserts only what holds by construction and the ranking gain."""
    exact = world["fom"]
    best = int(np.argmin(exact))
    fp, top = rank_all(trained["s"], world, 32)
    fp0, top0 = rank_all(trained["untrained"], world, 32)
    r1, r0 = spearman(fp, exact), spearman(fp0, exact)
    pos = int(np.nonzero(np.argsort(fp, kind="stable") == best)[0][0])
    near = int(np.sum(exact <= 1.15 * exact[best]))
    train_best = float(exact[np.nonzero(np.isin(np.arange(N_MAPS), np.random.default_rng(31).permutation(
        N_MAPS)[:4096]))[0]].min())
    s = make4(world, steps=0)
    s.set_params(trained["s"].get_params())
    found, n_exact, rnd_found = pruned_search(world, s)
    s.close()
    print(f"exhaustive optimum FoM {exact[best]:.6g} (map {best}, surrogate rank {pos}, {near} maps within 15 %); "
          f"best of the training maps {train_best:.6g}; surrogate top-32 best {exact[top].min():.6g}, untrained "
          f"top-32 best {exact[top0].min():.6g}; rank correlation trained {r1:.3f}, untrained {r0:.3f}; pruned "
          f"search best {found:.6g} after {n_exact} exact solves (round {rnd_found}) vs {N_MAPS}")
    assert found <= train_best
    assert r1 > r0 + 0.3


def move_set():
    """Every single and pair flip of the 16 cells (136 moves), CSR."""
    pairs = [(a,) for a in range(16)] + [(a, b) for a in range(16) for b in range(a + 1, 16)]
    off = np.zeros(len(pairs) + 1, np.int32)
    off[1:] = np.cumsum([len(q) for q in pairs])
    return off, np.concatenate(pairs).astype(np.int32)


K_VERIFY = 48


def test_pruned_search_matches_exhaustive_search(world, trained):
    """From four seeded starts, the search that solves only the surrogate's
    top 48 of the 136 single and pair flips per step (with the exact fallback),
    learning from every exact solve it makes, ends at the same FoM as the
    search that solves all 136, with fewer exact solves."""
    ev = world["ev"]
    s = make4(world, steps=0)
    s.set_params(trained["s"].get_params())

    def top_k(m, off, cells):
        fp = torch.zeros(len(off) - 1, dtype=torch.float64, device=DEV)
        top = torch.zeros(K_VERIFY, dtype=torch.int32, device=DEV)
        s.rank(ev, torch.from_numpy(m).to(DEV), torch.from_numpy(off).to(DEV), torch.from_numpy(cells).to(DEV),
               K_VERIFY, fp, top)
        torch.cuda.synchronize()
        return top.cpu().numpy()

    base_maps, base_target = world["train"]
    seen = {"maps": [], "target": []}

    def learn(maps, S):
        # every exact solve of the search joins the training set (online fine-tuning)
        seen["maps"].append(maps)
        seen["target"].append(pxd.Surrogate.encode(S, ENTRIES))
        new_m, new_t = np.concatenate(seen["maps"]), np.concatenate(seen["target"])
        rep = max(1, 2048 // len(new_m))
        train_more(s, np.concatenate([base_maps[:2048], np.tile(new_m, (rep, 1))]),
                   np.concatenate([base_target[:2048], np.tile(new_t, (rep, 1, 1))]), 40, seed=len(new_m))

    off, cells = move_set()
    tot_ex = tot_pr = 0
    for seed in range(4):
        start = ((np.random.default_rng(900 + seed).random(16)) < 0.5).astype(np.uint8)
        ex = descent(ev, start, off, cells, max_steps=40)
        pr = descent(ev, start, off, cells, max_steps=40, ranker=top_k, top_k=K_VERIFY, learn=learn)
        print(f"start {seed}: exhaustive {ex.fom:.6g} ({ex.exact_solves} exact solves), pruned {pr.fom:.6g} "
              f"({pr.exact_solves}; steps {[t[3] for t in pr.trace]})")
        assert pr.fom == ex.fom
        assert all(t[3] != "exhaustive" for t in pr.trace)
        tot_ex += ex.exact_solves
        tot_pr += pr.exact_solves
    s.close()
    assert tot_pr < tot_ex


def test_device_encoding_matches_host_encoding():
    """pxd_sur_encode forms the training targets on the device from S in the
    evaluator's layout: the same numbers as the host-side encode (float32
    rounding), tiny entries clamped at 1e-30 alike."""
    freqs = FREQS
    entries = ((0, 0), (1, 0), (2, 0), (2, 1))
    s = pxd.Surrogate(CFG.n_layers, CFG.ny, CFG.nx, freqs, freqs[0], freqs[-1], channels=CFG.channels,
                      hidden=CFG.hidden, emb=CFG.emb, entries=entries, precision=pxd.SUR_FP32, max_batch=8)
    rng = np.random.default_rng(3)
    n, P = 5, 3
    S = rng.normal(size=(n, len(freqs), P, P)) + 1j * rng.normal(size=(n, len(freqs), P, P))
    S[0, 0, 2, 1] = 0.0
    S *= np.exp(rng.uniform(-8, 0, size=S.shape))
    t_S = torch.from_numpy(np.ascontiguousarray(np.stack([S.real, S.imag], -1))).to(DEV)
    tgt = torch.empty((n, len(freqs), 3 * len(entries)), dtype=torch.float32, device=DEV)
    s.encode_device(t_S, tgt)
    torch.cuda.synchronize()
    ref = pxd.Surrogate.encode(S, entries)
    got = tgt.cpu().numpy()
    s.close()
    assert np.allclose(got, ref, rtol=1e-6, atol=1e-6), np.abs(got - ref).max()


# ---------------------------------------------------------------- fused inference

# (network, frequencies, max_batch): the 8 x 8 and working-size nets, a 32 x 32
# map (one workgroup per CU: 124 KB of LDS), and other channel orders with one
# and eight input planes (every row-tile count of a wave task from 1 to 5 occurs).
FUSED = [
    (osur.SurrogateConfig(n_layers=3, ny=8, nx=8, channels=(32, 32, 64, 64), hidden=64, emb=16, n_out=9), 7, 8),
    (osur.SurrogateConfig(n_layers=3, ny=24, nx=24, channels=(32, 32, 64, 64), hidden=256, emb=16, n_out=9), 101, 64),
    (osur.SurrogateConfig(n_layers=3, ny=32, nx=32, channels=(32, 32, 64, 64), hidden=256, emb=16, n_out=9), 21, 16),
    (osur.SurrogateConfig(n_layers=1, ny=16, nx=8, channels=(32, 64, 32, 64), hidden=32, emb=8, n_out=6), 5, 16),
    (osur.SurrogateConfig(n_layers=8, ny=8, nx=16, channels=(64, 32, 32, 32), hidden=128, emb=16, n_out=12), 9, 16),
]
ALL_ENTRIES = ((0, 0), (1, 0), (2, 0), (2, 1))


def fused_pair(cfg, freqs, max_batch):
    kw = dict(entries=ALL_ENTRIES[:cfg.n_out // 3], channels=cfg.channels, hidden=cfg.hidden, emb=cfg.emb,
              precision=pxd.SUR_BF16, max_batch=max_batch)
    f = pxd.Surrogate(cfg.n_layers, cfg.ny, cfg.nx, freqs, freqs[0], freqs[-1], **kw)
    g = pxd.Surrogate(cfg.n_layers, cfg.ny, cfg.nx, freqs, freqs[0], freqs[-1],
                      inference=pxd.SUR_INFER_GENERIC, **kw)
    return f, g


@pytest.mark.parametrize("i", range(len(FUSED)))
def test_fused_inference_matches_generic_and_oracle(i):
    """The fused kernels against the generic BF16 products and against the
    FP64 oracle (the BF16 bar above, 2e-2).  Both sides round the same
    operands to BF16 and sum in k order (on gfx950 they agree bit for bit);
    the bound allows for FP32 sums in another order, where an activation on
    either side of a BF16 rounding boundary rounds the other way (5e-3)."""
    cfg, F, mb = FUSED[i]
    freqs = np.linspace(2e9, 7e9, F)
    fu, ge = fused_pair(cfg, freqs, mb)
    assert fu.inference == pxd.SUR_INFER_FUSED and ge.inference == pxd.SUR_INFER_GENERIC
    p32 = init_params(cfg, 20 + i).astype(np.float32)
    fu.set_params(p32)
    ge.set_params(p32)
    B = min(mb, 5)
    maps = random_maps(B, cfg.n_layers * cfg.ny * cfg.nx, 30 + i)
    tm = torch.from_numpy(maps).to(DEV)
    outs = []
    for s in (fu, ge):
        o = torch.full((B, F, cfg.n_out), float("nan"), dtype=torch.float32, device=DEV)
        s.forward(tm, o)
        outs.append(o.cpu().numpy())
    want, _ = osur.forward(p32.astype(np.float64), maps, u_of(freqs), cfg)
    print(f"fused vs generic {rel(outs[0], outs[1]):.2e}, fused vs oracle {rel(outs[0], want):.2e}, "
          f"generic vs oracle {rel(outs[1], want):.2e}")
    assert np.isfinite(outs[0]).all()
    assert rel(outs[0], outs[1]) <= 5e-3
    assert rel(outs[0], want) <= 2e-2
    fu.close()
    ge.close()


def test_fused_inference_at_max_batch():
    """2,048 working-size maps in one call (2,048 trunk workgroups, 512 head
    blocks) against the generic products, per map."""
    cfg, F, _ = FUSED[1]
    freqs = np.linspace(1e9, 8e9, F)
    fu, ge = fused_pair(cfg, freqs, 2048)
    p32 = init_params(cfg, 40).astype(np.float32)
    fu.set_params(p32)
    ge.set_params(p32)
    maps = random_maps(2048, 3 * 24 * 24, 41, p=0.3)
    tm = torch.from_numpy(maps).to(DEV)
    outs = []
    for s in (fu, ge):
        o = torch.full((2048, F, 9), float("nan"), dtype=torch.float32, device=DEV)
        s.forward(tm, o)
        outs.append(o.cpu().numpy())
    per_map = np.array([rel(outs[0][b], outs[1][b]) for b in range(2048)])
    print(f"fused vs generic per map: max {per_map.max():.2e}, median {np.median(per_map):.2e}")
    assert np.isfinite(outs[0]).all() and per_map.max() <= 1e-2
    fu.close()
    ge.close()


SPEC8 = spec_variant("small6x3", n_layers=2, nx=8, ny=8, a=1e-3, n_freq=9, f_lo=3e9, f_hi=8e9, seed=33,
                     ports=(PortSpec("right", 0), PortSpec("top", 1), PortSpec("left", 0)))


def test_fused_ranking_is_the_fom_of_its_predictions():
    """pxd_sur_rank on the fused path (2 x 8 x 8 maps, every single flip and
    every pair of the first 24 cells, batches of 256): fom_pred against the
    FoM the oracle computes from the fused forward outputs of sampled
    candidates, top-k against a sort, and close to the generic path's fom_pred."""
    from oracle import fom as ofom

    freqs = SPEC8.freqs
    pb = pxd.Problem.from_spec(SPEC8)
    ev = pxd.Evaluator(precision=pxd.PREC_FP64)
    ev.load_parent(pb.fill(freqs, n_threads=16), freqs)
    ev.load_problem(pb, SPEC8.z0)
    ev.set_fom_paper()
    cfg = osur.SurrogateConfig(n_layers=2, ny=8, nx=8, channels=(32, 32, 64, 64), hidden=128, emb=16, n_out=12)
    fu, ge = fused_pair(cfg, freqs, 256)
    assert fu.inference == pxd.SUR_INFER_FUSED
    p32 = init_params(cfg, 50).astype(np.float32)
    fu.set_params(p32)
    ge.set_params(p32)
    n = 2 * 64
    iu, ju = np.triu_indices(24, 1)
    off = np.concatenate([np.arange(n + 1), n + 2 * np.arange(1, len(iu) + 1)]).astype(np.int32)
    cells = np.concatenate([np.arange(n), np.stack([iu, ju], 1).ravel()]).astype(np.int32)
    C = len(off) - 1
    base = SPEC8.base_map()
    fps = []
    for s in (fu, ge):
        fp = torch.zeros(C, dtype=torch.float64, device=DEV)
        top = torch.zeros(16, dtype=torch.int32, device=DEV)
        s.rank(ev, torch.from_numpy(base).to(DEV), torch.from_numpy(off).to(DEV), torch.from_numpy(cells).to(DEV),
               16, fp, top)
        torch.cuda.synchronize()
        fps.append((fp.cpu().numpy(), top.cpu().numpy()))
    fp, top = fps[0]
    assert np.array_equal(top, np.argsort(fp, kind="stable")[:16])
    assert np.max(np.abs(fp - fps[1][0]) / fps[1][0]) <= 5e-2
    pick = np.array([0, 1, 127, 128, C - 1, int(top[0])])
    maps = np.repeat(base[None], len(pick), 0)
    for r, c in enumerate(pick):
        maps[r, cells[off[c]:off[c + 1]]] ^= 1
    out = torch.zeros((len(pick), len(freqs), 12), dtype=torch.float32, device=DEV)
    fu.forward(torch.from_numpy(maps).to(DEV), out)
    o = out.cpu().numpy().astype(np.float64)
    for r in range(len(pick)):
        S = np.zeros((len(freqs), 3, 3), np.complex128)
        for e, (i, j) in enumerate(ALL_ENTRIES):
            S[:, i, j] = np.exp(o[r, :, 3 * e])
        assert abs(ofom.fom(S, freqs) - fp[pick[r]]) <= 1e-9 * fp[pick[r]]
    fu.close()
    ge.close()
    ev.close()
