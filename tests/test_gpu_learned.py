"""GPU learned heavy-pair seeding against the fp64 oracle (oracle/learned.py).

Integer work (prefix statistics behind the features, candidate pairs, label
lookup, seed selection) is compared exactly.  Floating point:

* features: fp32 logs/divisions of exact integers, relative 1e-5 (atol 1e-6);
* gradients: fp32 sums of at most 128 products per entry; each tensor within
  1e-4 of its largest oracle entry (the fp32 sum of N terms errs by about
  N * 2^-24 of the summed magnitudes);
* Adam: the update formula checked exactly (relative 1e-5 of the step size)
  given the GPU's own gradient, and a three-step trajectory against the pure
  oracle within a few per mille of the step size;
* bf16 scores: against the oracle forward on bf16-rounded weights and inputs,
  1e-4 * (max |score| + 1); against the fp32 forward, an RMS difference of at
  most 1% of the RMS score.
"""
import numpy as np
import pytest

import datagen
import oracle
from oracle import learned as L

pytestmark = pytest.mark.gpu

SEED = 0x243F6A8885A308D3
KEYS = ("W1", "b1", "W2", "b2", "w3", "b3")
SHAPES = dict(W1=(64, 32), b1=(64,), W2=(64, 64), b2=(64,), w3=(64,), b3=(1,))


@pytest.fixture(scope="module")
def crop():
    import paper_1210_0461_amd as crop
    return crop


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


@pytest.fixture
def ctx(crop, torch):
    # the library works on torch's stream, so torch reads of its outputs are
    # ordered after its kernels
    h = crop.crop_create(0)
    crop.crop_set_stream(h, torch.cuda.current_stream())
    yield h
    crop.crop_synchronize(h)
    crop.crop_destroy(h)


def load(crop, ctx, st, P=8, seed=SEED):
    crop.crop_set_partitions(ctx, P)
    crop.crop_set_seed(ctx, seed)
    crop.crop_load_transactions(ctx, st.off, st.items, st.n)


def unflat(flat):
    out, k = {}, 0
    for name in KEYS:
        n = int(np.prod(SHAPES[name]))
        out[name] = np.asarray(flat[k:k + n], np.float64).reshape(SHAPES[name])
        k += n
    return out


def flat(d):
    return np.concatenate([np.asarray(d[k], np.float64).reshape(-1) for k in KEYS])


def rand_inputs(seed, N, scale=1.0):
    r = datagen.Raw(seed)
    Z = ((r.uniform(N * 32) * 2.0 - 1.0) * scale).reshape(N, 32).astype(np.float32)
    y = (r.uniform(N) * 4.0).astype(np.float32)
    return Z, y


# ---------------------------------------------------------------- features

@pytest.mark.parametrize("which,Tp", [("small", "prefix"), ("small", "all"), ("small", 0),
                                      ("small", 1), ("large", "prefix")])
def test_item_features(crop, ctx, torch, which, Tp):
    st = datagen.config_small() if which == "small" else datagen.config_large()
    Tp = L.prefix_len(st.T) if Tp == "prefix" else (st.T if Tp == "all" else Tp)
    print(f"features {which} T={st.T} Tp={Tp}", flush=True)
    load(crop, ctx, st)
    feat = torch.empty((st.n, 16), dtype=torch.float32, device="cuda")
    crop.crop_item_features(ctx, Tp, feat)
    got = feat.cpu().numpy().astype(np.float64)
    want = L.item_features(L.item_stats(st.off, st.items, st.n, Tp), Tp)
    np.testing.assert_allclose(got, want, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("M", [2, 3, 57, 200, 500])
def test_top_item_pairs(crop, ctx, torch, M):
    st = datagen.config_small()   # n = 500, many tied prefix counts
    Tp = L.prefix_len(st.T)
    load(crop, ctx, st)
    n_pairs = M * (M - 1) // 2
    cx = torch.full((n_pairs + 5,), -1, dtype=torch.int32, device="cuda")
    cy = torch.full((n_pairs + 5,), -1, dtype=torch.int32, device="cuda")
    got_n = crop.crop_top_item_pairs(ctx, Tp, M, cx, cy)
    assert got_n == n_pairs
    st_o = L.item_stats(st.off, st.items, st.n, Tp)
    _, ex, ey = L.candidates(st_o["A"], M)
    np.testing.assert_array_equal(cx.cpu().numpy()[:n_pairs].astype(np.uint32), ex)
    np.testing.assert_array_equal(cy.cpu().numpy()[:n_pairs].astype(np.uint32), ey)
    assert (cx.cpu().numpy()[n_pairs:] == -1).all()   # nothing written past the pairs


def test_top_item_pairs_rejects(crop, ctx, torch):
    st = datagen.config_small()
    load(crop, ctx, st)
    cx = torch.empty(10, dtype=torch.int32, device="cuda")
    with pytest.raises(crop.CropError) as e:
        crop.crop_top_item_pairs(ctx, 100, 6, cx, cx)      # 15 pairs > capacity 10
    assert e.value.status == -4
    with pytest.raises(crop.CropError):
        crop.crop_top_item_pairs(ctx, 100, st.n + 1, cx, cx)
    with pytest.raises(crop.CropError):
        crop.crop_item_features(ctx, st.T + 1, torch.empty((st.n, 16), device="cuda"))


# ---------------------------------------------------------------- labels

@pytest.mark.parametrize("case", ["small", "wide"])
def test_lookup_exact(crop, ctx, torch, case):
    if case == "small":
        st, P = datagen.config_small(), 8
    else:   # item ids beyond 16 bits: the 64-bit key layout
        st, P = datagen.tiny_transactions(77, T=300, n=200_000, zipf_s=0.6, mean_len=6,
                                          cap=20), 4
    load(crop, ctx, st, P)
    crop.crop_run_exact(ctx)
    r = oracle.tx_exact(st.off, st.items, P, SEED)
    present = dict(zip(oracle.pack_keys(r["x"], r["y"]).tolist(), r["cnt"].tolist()))
    rng = datagen.Raw(91)
    k = min(2000, r["x"].shape[0])
    pick = rng.randint(k, 0, r["x"].shape[0] - 1)
    qx = list(r["x"][pick])
    qy = list(r["y"][pick])
    # absent pairs
    ax = rng.randint(500, 0, st.n - 2)
    ay = ax + 1 + rng.randint(500, 0, 3)
    ay = np.minimum(ay, st.n - 1)
    qx += list(ax)
    qy += list(ay)
    qx = np.array(qx, np.uint32)
    qy = np.array(qy, np.uint32)
    want = np.array([present.get((int(a) << 32) | int(b), 0) for a, b in zip(qx, qy)],
                    np.int64)
    tq = lambda a: torch.from_numpy(a.astype(np.int32)).cuda()
    out = torch.full((qx.shape[0],), -1, dtype=torch.int32, device="cuda")
    crop.crop_lookup_exact(ctx, tq(qx), tq(qy), out)
    np.testing.assert_array_equal(out.cpu().numpy().astype(np.int64), want)
    assert (want == 0).any() and (want > 0).any()


def test_pair_inputs(crop, ctx, torch):
    st = datagen.config_small()
    load(crop, ctx, st)
    Tp = L.prefix_len(st.T)
    feat = torch.empty((st.n, 16), dtype=torch.float32, device="cuda")
    crop.crop_item_features(ctx, Tp, feat)
    rng = datagen.Raw(5)
    cx = rng.randint(777, 0, st.n - 1).astype(np.int32)
    cy = rng.randint(777, 0, st.n - 1).astype(np.int32)
    cnt = rng.randint(777, 0, 100000).astype(np.int32)
    Z = torch.empty((777, 32), dtype=torch.float32, device="cuda")
    y = torch.empty(777, dtype=torch.float32, device="cuda")
    tq = lambda a: torch.from_numpy(a).cuda()
    crop.crop_pair_inputs(ctx, feat, tq(cx), tq(cy), tq(cnt), Z, y)
    f = feat.cpu().numpy()
    np.testing.assert_array_equal(Z.cpu().numpy(), np.concatenate([f[cx], f[cy]], axis=1))
    np.testing.assert_allclose(y.cpu().numpy(), np.log1p(cnt.astype(np.float64)), rtol=3e-7)


# ---------------------------------------------------------------- network

@pytest.mark.parametrize("N,wseed", [(128, 11), (37, 12), (1, 13)])
def test_mlp_grad(crop, ctx, torch, N, wseed):
    w = datagen.mlp_init_weights(wseed)
    from paper_1210_0461_amd.seeding import flat_init
    mlp = crop.crop_mlp_create(ctx, flat_init(w))
    try:
        Z, y = rand_inputs(wseed + 100, N)
        g, loss = crop.crop_mlp_grad(ctx, mlp, torch.from_numpy(Z).cuda(),
                                     torch.from_numpy(y).cuda())
        want_loss, want = L.mlp_backward({k: w[k] for k in KEYS}, Z, y)
        assert abs(loss - want_loss) <= 1e-5 * (abs(want_loss) + 1e-3)
        got = unflat(g)
        for k in KEYS:
            scale = np.abs(want[k]).max()
            np.testing.assert_allclose(got[k], want[k].reshape(SHAPES[k]), rtol=0,
                                       atol=1e-4 * scale + 1e-9, err_msg=k)
        # the weights are unchanged by a gradient call
        np.testing.assert_array_equal(crop.crop_mlp_params(ctx, mlp), flat_init(w))
    finally:
        crop.crop_mlp_destroy(mlp)


def test_mlp_adam_update(crop, ctx, torch):
    """Two single Adam steps, each checked against the oracle's update from the
    GPU's own gradient and the moments carried along by the oracle."""
    from paper_1210_0461_amd.seeding import flat_init
    w = datagen.mlp_init_weights(21)
    mlp = crop.crop_mlp_create(ctx, flat_init(w))
    try:
        Z, y = rand_inputs(121, 64)
        tZ, ty = torch.from_numpy(Z).cuda(), torch.from_numpy(y).cuda()
        order = torch.arange(64, dtype=torch.int32, device="cuda")
        p = {k: v for k, v in unflat(flat_init(w)).items()}
        m = {k: np.zeros(SHAPES[k]) for k in KEYS}
        v = {k: np.zeros(SHAPES[k]) for k in KEYS}
        lr = 1e-2
        for t in (1, 2):
            g, _ = crop.crop_mlp_grad(ctx, mlp, tZ, ty)
            crop.crop_mlp_train(ctx, mlp, tZ, ty, order, 64, lr)
            p, m, v = L.adam_step(p, unflat(g), m, v, t, lr=lr)
            got = crop.crop_mlp_params(ctx, mlp)
            np.testing.assert_allclose(got, flat(p), rtol=0, atol=1e-5 * lr + 1e-7)
            p = unflat(got)   # continue from the GPU's fp32 weights
    finally:
        crop.crop_mlp_destroy(mlp)


def test_mlp_train_trajectory(crop, ctx, torch):
    """Three minibatch steps through crop_mlp_train (one launch) against the
    oracle's own gradient and Adam steps in fp64; a ragged final batch is
    ignored."""
    from paper_1210_0461_amd.seeding import flat_init
    w = datagen.mlp_init_weights(31)
    mlp = crop.crop_mlp_create(ctx, flat_init(w))
    try:
        Z, y = rand_inputs(131, 300)
        order = datagen.sample_order(7, 300, 2)[:3 * 96 + 50]
        crop.crop_mlp_train(ctx, mlp, torch.from_numpy(Z).cuda(), torch.from_numpy(y).cuda(),
                            torch.from_numpy(order.astype(np.int32)).cuda(), 96, 3e-3)
        got = crop.crop_mlp_params(ctx, mlp)
        p = {k: np.asarray(w[k], np.float64) for k in KEYS}
        m = {k: np.zeros(SHAPES[k]) for k in KEYS}
        v = {k: np.zeros(SHAPES[k]) for k in KEYS}
        for t in range(1, 4):
            idx = order[(t - 1) * 96:t * 96]
            loss, g = L.mlp_backward(p, Z[idx], y[idx])
            p, m, v = L.adam_step(p, g, m, v, t, lr=3e-3)
        step = np.abs(flat(p) - flat({k: w[k] for k in KEYS}))
        diff = np.abs(got - flat(p))
        assert diff.max() <= 3 * 3e-3 * 5e-3 + 1e-7, diff.max()
        assert step.max() > 1e-3   # the steps moved the weights
        assert abs(crop.crop_mlp_loss(ctx, mlp) - loss) <= 1e-3 * loss + 1e-5
    finally:
        crop.crop_mlp_destroy(mlp)


@pytest.mark.parametrize("N", [1, 255, 4099])
def test_mlp_score_bf16(crop, ctx, torch, N):
    from paper_1210_0461_amd.seeding import flat_init
    w = datagen.mlp_init_weights(41)
    w["b1"] = (np.arange(64, dtype=np.float32) - 32) / 64
    w["b3"] = np.array([0.3], np.float32)
    mlp = crop.crop_mlp_create(ctx, flat_init(w))
    try:
        Z, _ = rand_inputs(141, N, scale=3.0)
        out = torch.empty(N, dtype=torch.float32, device="cuda")
        crop.crop_mlp_score(ctx, mlp, torch.from_numpy(Z).cuda(), out)
        got = out.cpu().numpy().astype(np.float64)
        want_bf = L.mlp_score_bf16(w, Z)
        # the GPU sums in fp32, the oracle in fp64: an activation that lies
        # at a bfloat16 rounding boundary can round the other way (about one
        # in 2^16), moving its sample's score by one bfloat16 step of that
        # activation's contribution; every other sample agrees to fp32 sums
        err = np.abs(got - want_bf)
        scale = np.abs(want_bf).max() + 1
        assert np.quantile(err, 0.99) <= 1e-4 * scale, err.max()
        assert err.max() <= 1e-2 * scale, err.max()
        # bf16 rounding (relative 2^-9 per weight, input and activation)
        # costs about a per mille of the score's scale against the fp32
        # network
        want_32, _ = L.mlp_forward({k: w[k] for k in KEYS}, Z)
        rms = lambda a: float(np.sqrt(np.mean(np.square(a))))
        assert rms(got - want_32) <= 1e-2 * (rms(want_32) + 1e-3), rms(got - want_32)
    finally:
        crop.crop_mlp_destroy(mlp)


@pytest.mark.parametrize("n,R", [(1, 1), (1000, 0), (1000, 17), (5000, 5000)])
def test_select_seeds(crop, ctx, torch, n, R):
    rng = datagen.Raw(n + R)
    score = (np.floor(rng.uniform(n) * 50) / 7).astype(np.float32)   # many ties
    cx = np.arange(n, dtype=np.int32)
    cy = np.arange(n, dtype=np.int32) + 1
    sx = torch.full((R + 3,), -1, dtype=torch.int32, device="cuda")
    sy = torch.full((R + 3,), -1, dtype=torch.int32, device="cuda")
    tq = lambda a: torch.from_numpy(a).cuda()
    crop.crop_select_seeds(ctx, tq(score), tq(cx), tq(cy), R, sx, sy)
    order = np.lexsort((np.arange(n), -score.astype(np.float64)))[:R]
    np.testing.assert_array_equal(sx.cpu().numpy()[:R], cx[order])
    np.testing.assert_array_equal(sy.cpu().numpy()[:R], cy[order])
    assert (sx.cpu().numpy()[R:] == -1).all()


# ---------------------------------------------------------------- end to end

def test_seeding_pipeline_small(crop, ctx, torch):
    """Train on two small streams, seed a third, run seeded Space-Saving: every
    pinned pair must be counted exactly (zero error) and the run must satisfy
    the Section 4 invariants checked elsewhere; recall is reported, not
    asserted."""
    from paper_1210_0461_amd import seeding
    streams = [datagen.transactions(20_000, 2000, 1.1, 8.0, 32, datagen.Raw(900 + i), "s")
               for i in range(3)]
    P, M = 4, 48
    Zs, ys = [], []
    for st in streams[:2]:
        load(crop, ctx, st, P)
        Z, y, cx, cy, sup = seeding.training_pairs(ctx, st.T, st.n, M)
        # labels against the oracle's exact counts
        r = oracle.tx_exact(st.off, st.items, 1, SEED)
        cnt = dict(zip(oracle.pack_keys(r["x"], r["y"]).tolist(), r["cnt"].tolist()))
        hx, hy = cx.cpu().numpy().astype(np.int64), cy.cpu().numpy().astype(np.int64)
        want = np.array([cnt.get((a << 32) | b, 0) for a, b in zip(hx, hy)])
        np.testing.assert_array_equal(sup.cpu().numpy(), want)
        Zs.append(Z)
        ys.append(y)
    Z = torch.cat(Zs)
    y = torch.cat(ys)
    mlp = crop.crop_mlp_create(ctx, seeding.flat_init(datagen.mlp_init_weights(1)))
    try:
        order = torch.from_numpy(datagen.sample_order(3, Z.shape[0], 4).astype(np.int32)).cuda()
        crop.crop_mlp_train(ctx, mlp, Z, y, order, 128, 3e-3)
        loss = crop.crop_mlp_loss(ctx, mlp)
        assert np.isfinite(loss)
        st = streams[2]
        load(crop, ctx, st, P)
        sx, sy, score = seeding.predict_seeds(ctx, mlp, st.T, st.n, M, 64)
        crop.crop_set_summary(ctx, 256, 8)
        crop.crop_run_topk_seeded(ctx, 100, sx, sy, 4)
        s = crop.crop_read_summary(ctx, P * 256)
        r = oracle.tx_exact(st.off, st.items, 1, SEED)
        cnt = dict(zip(oracle.pack_keys(r["x"], r["y"]).tolist(), r["cnt"].tolist()))
        pinned = s["pinned"]
        assert pinned.any()
        for a, b, c, e in zip(s["x"][pinned], s["y"][pinned], s["cnt"][pinned],
                              s["err"][pinned]):
            assert e == 0 and c == cnt.get((int(a) << 32) | int(b), 0)
    finally:
        crop.crop_mlp_destroy(mlp)


def test_mlp_train_rejects_bad_index(crop, ctx, torch):
    from paper_1210_0461_amd.seeding import flat_init
    w = datagen.mlp_init_weights(51)
    mlp = crop.crop_mlp_create(ctx, flat_init(w))
    try:
        Z, y = rand_inputs(151, 40)
        order = np.arange(64, dtype=np.int32) % 40
        order[50] = 40                                     # one past the samples
        with pytest.raises(crop.CropError) as e:
            crop.crop_mlp_train(ctx, mlp, torch.from_numpy(Z).cuda(),
                                torch.from_numpy(y).cuda(),
                                torch.from_numpy(order).cuda(), 32, 1e-3)
        assert e.value.status == -3
        np.testing.assert_array_equal(crop.crop_mlp_params(ctx, mlp), flat_init(w))
        with pytest.raises(crop.CropError):
            crop.crop_mlp_grad(ctx, mlp, torch.from_numpy(Z).cuda()[:0],
                               torch.from_numpy(y).cuda()[:0])
    finally:
        crop.crop_mlp_destroy(mlp)


def test_seeded_run_rejects_invalid_seed_pairs(crop, ctx, torch):
    """Seeds must be pairs x < y < n_items: an unordered pair, a diagonal
    pair or an id beyond the stream's items is reported with its index and
    nothing runs; valid seeds still run afterwards."""
    st = datagen.config_small()
    load(crop, ctx, st, 8)
    crop.crop_set_summary(ctx, 256, 8)
    good_x = np.array([1, 2, 3, 4], np.int32)
    good_y = np.array([5, 6, 7, 8], np.int32)
    for k, (x, y) in enumerate([(9, 3), (7, 7), (2, st.n), (0, 1 << 20)]):
        sx = good_x.copy()
        sy = good_y.copy()
        sx[2], sy[2] = x, y
        with pytest.raises(crop.CropError) as e:
            crop.crop_run_topk_seeded(ctx, 10, torch.from_numpy(sx).cuda(),
                                      torch.from_numpy(sy).cuda(), 4)
        assert e.value.status == -3 and e.value.index == 2, (k, e.value)
    crop.crop_run_topk_seeded(ctx, 10, torch.from_numpy(good_x).cuda(),
                              torch.from_numpy(good_y).cuda(), 4)
    s = crop.crop_read_summary(ctx, 8 * 256)
    assert int(s["pinned"].sum()) == 4


def test_seeding_gain_over_plain_summary(crop, ctx, torch):
    """What the trained network adds at equal memory: six training streams
    and one held-out stream of 200,000 transactions (like the 1M-transaction
    workload, other seeds), one partition of 4,096 counters (ell = 16) and
    the top 200 by guaranteed count.  Seeded recall and count error must be
    at least as good as the plain summary's; pinned pairs carry their exact
    supports."""
    from paper_1210_0461_amd import seeding
    mk = lambda seed: datagen.transactions(200_000, 50_000, 1.1, 10.0, 64, datagen.Raw(seed),
                                           "g")
    P, M, K, R = 64, 128, 200, 256
    Zs, ys = [], []
    for i in range(6):
        st = mk(7000 + i)
        load(crop, ctx, st, P)
        Z, y, _, _, _ = seeding.training_pairs(ctx, st.T, st.n, M)
        Zs.append(Z)
        ys.append(y)
    Z, y = torch.cat(Zs), torch.cat(ys)
    mlp = crop.crop_mlp_create(ctx, seeding.flat_init(datagen.mlp_init_weights(2)))
    try:
        order = torch.from_numpy(datagen.sample_order(8, Z.shape[0], 8).astype(np.int32)).cuda()
        crop.crop_mlp_train(ctx, mlp, Z, y, order, 128, 1e-3)
        st = mk(7100)
        ref = oracle.tx_exact(st.off, st.items, 1, SEED)
        rk = oracle.pack_keys(ref["x"], ref["y"])
        exact = dict(zip(rk.tolist(), ref["cnt"].tolist()))
        load(crop, ctx, st, 1)
        sx, sy, _ = seeding.predict_seeds(ctx, mlp, st.T, st.n, M, R)
        crop.crop_set_summary(ctx, 4096, 16)
        res = {}
        for mode in ("plain", "seeded"):
            if mode == "plain":
                crop.crop_run_topk(ctx, K)
            else:
                crop.crop_run_topk_seeded(ctx, K, sx, sy, 4)
            i, j, up, lo, _ = crop.crop_read_topk(ctx, K)
            keys = oracle.pack_keys(i, j)
            truth = np.array([exact[int(k)] for k in keys], np.float64)
            res[mode] = dict(recall=oracle.recall_at_k(keys, rk, ref["cnt"], K),
                             err=float((up - truth).max()), gap=float((truth - lo).max()))
            if mode == "seeded":
                s = crop.crop_read_summary(ctx, 4096)
                pk = oracle.pack_keys(s["x"], s["y"])
                for q in np.flatnonzero(s["pinned"]):
                    assert s["cnt"][q] == exact.get(int(pk[q]), 0) and s["err"][q] == 0
        print(f"plain {res['plain']}  seeded {res['seeded']}", flush=True)
        assert res["seeded"]["recall"] >= res["plain"]["recall"]
        assert res["seeded"]["gap"] <= res["plain"]["gap"]
    finally:
        crop.crop_mlp_destroy(mlp)


def _fisher_yates_order(seed, n, epochs):
    """The predictor's minibatch order, restated: one Fisher-Yates
    permutation per epoch driven by SplitMix64, j = (word * (i + 1)) >> 64."""
    m64 = (1 << 64) - 1
    s = seed & m64
    out = []
    for _ in range(epochs):
        p = list(range(n))
        for i in range(n - 1, 0, -1):
            s = (s + 0x9E3779B97F4A7C15) & m64
            z = s
            z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m64
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m64
            z ^= z >> 31
            j = (z * (i + 1)) >> 64
            p[i], p[j] = p[j], p[i]
        out += p
    return np.array(out, np.int32)


def test_predictor_object_matches_stepwise_calls(crop, ctx, torch):
    """crop_predictor_train / score / free give exactly what the step-wise
    calls give with the same inputs: the same trained weights (labels from
    exact runs, the same minibatch order) and the same seeds."""
    from paper_1210_0461_amd import seeding
    streams = [datagen.transactions(20000, 3000, 1.1, 10.0, 64, datagen.Raw(7100 + k), f"p{k}")
               for k in range(3)]
    M, epochs, bs, lr, sseed = 64, 2, 128, 3e-3, 99
    init = seeding.flat_init(datagen.mlp_init_weights(17))
    crop.crop_set_partitions(ctx, 16)
    crop.crop_set_seed(ctx, SEED)
    held = datagen.transactions(20000, 3000, 1.1, 10.0, 64, datagen.Raw(7200), "held")
    crop.crop_load_transactions(ctx, held.off, held.items, held.n)
    pred = crop.crop_predictor_train(ctx, [(s.off, s.items, s.n) for s in streams],
                                     top_items=M, epochs=epochs, batch=bs, lr=lr,
                                     shuffle_seed=sseed, init=init)
    try:
        # the caller's loaded stream is untouched: an exact run still works on it
        crop.crop_run_exact(ctx)
        w_obj, loss_obj = crop.crop_predictor_params(ctx, pred)
        # step-wise
        Zs, ys = [], []
        for s in streams:
            crop.crop_load_transactions(ctx, s.off, s.items, s.n)
            Z, y, _, _, _ = seeding.training_pairs(ctx, s.T, s.n, M)
            Zs.append(Z)
            ys.append(y)
        Z = torch.cat(Zs)
        y = torch.cat(ys)
        order = torch.from_numpy(_fisher_yates_order(sseed, Z.shape[0], epochs)).cuda()
        mlp = crop.crop_mlp_create(ctx, init)
        try:
            crop.crop_mlp_train(ctx, mlp, Z, y, order, bs, lr)
            w_step = crop.crop_mlp_params(ctx, mlp)
            np.testing.assert_array_equal(w_obj, w_step)
            assert loss_obj == crop.crop_mlp_loss(ctx, mlp)
            crop.crop_load_transactions(ctx, held.off, held.items, held.n)
            R = 50
            sx = torch.zeros(R, dtype=torch.int32, device="cuda")
            sy = torch.zeros(R, dtype=torch.int32, device="cuda")
            n = crop.crop_predictor_score(ctx, pred, R, sx, sy)
            assert n == R
            tx, ty, _ = seeding.predict_seeds(ctx, mlp, held.T, held.n, M, R)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(sx.cpu().numpy(), tx.cpu().numpy())
            np.testing.assert_array_equal(sy.cpu().numpy(), ty.cpu().numpy())
            assert np.all(sx.cpu().numpy() < sy.cpu().numpy())
        finally:
            crop.crop_mlp_destroy(mlp)
    finally:
        crop.crop_predictor_free(pred)
    with pytest.raises(crop.CropError):
        crop.crop_predictor_train(ctx, [], top_items=M)


@pytest.mark.timeout(900)
def test_learned_seeding_at_full_size(crop, ctx, torch):
    """The learned workload at its stated size: the predictor is trained on
    the exact supports of 20 streams of 1M transactions (seeds 5000-5019,
    through crop_predictor_train) and seeds the held-out stream (seed 5100)
    with its 1,000 best candidate pairs (r_max 4).  At equal memory -- one
    partition of 16,384 counters, and 1,024 partitions of 2^14 counters,
    16 per bucket -- the seeded top-1000 recalls at least as many of the
    oracle's true top 1,000 as the plain summary in the library's default
    report order, and its largest gap between reported guaranteed count and
    exact support is no larger."""
    import time
    t0 = time.perf_counter()
    train = [datagen.config_learned_train(i) for i in range(20)]
    held = datagen.config_learned_heldout()
    print(f"generated 21 streams in {time.perf_counter() - t0:.1f} s", flush=True)
    crop.crop_set_seed(ctx, SEED)
    crop.crop_set_partitions(ctx, 1024)
    pred = crop.crop_predictor_train(ctx, [(s.off, s.items, s.n) for s in train],
                                     top_items=256, epochs=4, batch=128, lr=1e-3,
                                     shuffle_seed=6000)
    del train
    try:
        _, loss = crop.crop_predictor_params(ctx, pred)
        assert np.isfinite(loss)
        t0 = time.perf_counter()
        ref = oracle.tx_exact(held.off, held.items, 1, SEED)
        print(f"oracle on the held-out stream: {time.perf_counter() - t0:.1f} s", flush=True)
        rk = oracle.pack_keys(ref["x"], ref["y"])
        order = np.argsort(rk)
        rk, rc = rk[order], ref["cnt"][order].astype(np.int64)
        K = 1000
        crop.crop_load_transactions(ctx, held.off, held.items, held.n)
        sx = torch.zeros(K, dtype=torch.int32, device="cuda")
        sy = torch.zeros(K, dtype=torch.int32, device="cuda")
        assert crop.crop_predictor_score(ctx, pred, K, sx, sy) == K
        for P, C in ((1, 16384), (1024, 1 << 14)):
            crop.crop_set_partitions(ctx, P)
            crop.crop_set_summary(ctx, C, 16)
            res = {}
            for mode in ("plain", "seeded"):
                if mode == "plain":
                    crop.crop_run_topk(ctx, K)
                else:
                    crop.crop_run_topk_seeded(ctx, K, sx, sy, 4)
                i, j, up, lo, _ = crop.crop_read_topk(ctx, K)
                keys = oracle.pack_keys(i, j)
                pos = np.minimum(np.searchsorted(rk, keys), rk.shape[0] - 1)
                truth = np.where(rk[pos] == keys, rc[pos], 0)
                res[mode] = dict(recall=oracle.recall_at_k(keys, rk, rc, K),
                                 err=float((up - truth).max()),
                                 gap=float((truth - lo).max()))
            print(f"P={P} C={C}: plain {res['plain']} seeded {res['seeded']}", flush=True)
            assert res["seeded"]["recall"] >= res["plain"]["recall"]
            assert res["seeded"]["gap"] <= res["plain"]["gap"]
    finally:
        crop.crop_predictor_free(pred)
