"""Launch-shape autotuner for libtsvd.

The library's kernels take their launch shapes from the context's tuning
(tsvd_ctx_set_tuning): the BF16X3 Gram tile edge, the split-K chunk count, the
power launch's workgroup count, and, for batches, the team size rule and the
batched Gram's work-unit shape (tile edge and chunk length) per Gram-dimension
class.  None of these changes what is computed (the Gram's chunk order changes
FP32 rounding only); they change speed.

The tuner measures candidates per *shape class* through the public entry
points, with HIP events on the caller's stream, keeps the fastest, and stores
the choice in a JSON cache so later processes reuse it:

    tuner = Tuner(ctx, cache_path)
    tuner.tune_dense(A, gram="bf16x3", k=8)     # measures, stores
    tuner.apply_dense(m, n, "bf16x3")           # sets the stored tuning
    tuner.tune_batch(problems)                  # team_kib / group_kchunk
    tuner.tune_gram_classes(shapes)             # batched Gram unit per class
    tuner.apply_batch(shapes)                   # both, for a batch

A shape class buckets the Gram dimension d and the contraction length K to
powers of two (and the Gram mode and side), so that one measurement serves
every shape that would pick the same tiles.
"""

from __future__ import annotations

import json
import math
import os
import time

from . import GRAM_CLASSES, Context, gram_class, get_tuning, set_tuning

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2208_08410_amd", "tuning.json")


def _pow2_bucket(x: int) -> int:
    return 1 << max(0, int(math.ceil(math.log2(max(1, int(x))))))


def dense_class(m: int, n: int, gram: str, branch: int = 0) -> str:
    """Shape-class key of a single dense problem."""
    right = (m > n) if branch == 1 else (m >= n)
    d, K = (n, m) if right else (m, n)
    return f"dense/{gram}/{'R' if right else 'L'}/d{_pow2_bucket(d)}/K{_pow2_bucket(K)}"


def batch_class(shapes) -> str:
    """Shape-class key of a batch: problem count and the largest Gram, bucketed."""
    dmax = max(min(m, n) for m, n in shapes) if shapes else 1
    return f"batch/c{_pow2_bucket(len(shapes))}/d{_pow2_bucket(dmax)}"


def gram_candidates(gram: str, d: int, K: int, num_cu: int):
    """(gram_tile, gram_chunks) pairs worth measuring for one class."""
    tiles = [128, 256] if gram == "bf16x3" and d >= 256 else [0]
    out = []
    for t in tiles:
        bm = t or 128
        nt = (d + bm - 1) // bm
        T = nt * (nt + 1) // 2
        chunks = {0}
        for per_cu in (1, 2, 4, 8):
            s = max(1, (per_cu * num_cu + T - 1) // T)
            s = min(s, max(1, K // 256))
            chunks.add(int(s))
        out += [(t, c) for c in sorted(chunks)]
    return out


def power_candidates(d: int, num_cu: int):
    c = {0}
    for g in (num_cu // 4, num_cu // 2, 3 * num_cu // 4):
        if g >= 1 and g * 4 <= d:
            c.add(int(g))
    return sorted(c)


def batch_candidates():
    return [(tk, kc) for tk in (64, 128, 256, 512, 1024) for kc in (1024, 2048, 4096)]


def gram_unit_key(cls: int) -> str:
    """Cache key of a Gram-dimension class's batched unit shape."""
    return f"gram_unit/c{int(cls)}"


def gram_unit_candidates(K_max: int):
    """(tile edge, chunk rows) pairs of the batched Gram's work unit for a
    class whose longest contraction is K_max: chunk lengths past 2 K_max all
    give one chunk and are left out."""
    kcs = [kc for kc in (512, 1024, 2048, 4096, 8192) if kc <= max(512, 2 * int(K_max))]
    return [(t, kc) for t in (64, 128) for kc in kcs]


class Tuner:
    def __init__(self, ctx: Context, cache_path: str | None = None, reps: int = 3):
        self.ctx = ctx
        self.path = cache_path or DEFAULT_CACHE
        self.reps = int(reps)
        self.table = {}
        if os.path.exists(self.path):
            with open(self.path) as f:
                self.table = json.load(f)

    # ---- cache
    def save(self):
        os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.table, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def lookup(self, key: str):
        e = self.table.get(key)
        return dict(e["tuning"]) if e else None

    def apply(self, key: str) -> bool:
        """Set the stored tuning of `key` on the context (library defaults if
        the class was never tuned), with every class's stored batched-Gram
        unit shape.  Returns whether an entry was found."""
        t = self.lookup(key)
        merged = dict(t or {})
        merged.update(self.class_tuning())
        set_tuning(self.ctx, **merged)
        return t is not None

    def apply_dense(self, m: int, n: int, gram: str, branch: int = 0) -> bool:
        return self.apply(dense_class(m, n, gram, branch))

    def class_tuning(self) -> dict:
        """The stored batched-Gram unit shapes of every class, as the
        group_tile / group_kchunk_cls arguments of set_tuning (0 = library
        choice for classes never tuned)."""
        tiles, kcs = [0] * GRAM_CLASSES, [0] * GRAM_CLASSES
        for c in range(GRAM_CLASSES):
            e = self.lookup(gram_unit_key(c))
            if e:
                tiles[c], kcs[c] = int(e["group_tile"]), int(e["group_kchunk"])
        return {"group_tile": tiles, "group_kchunk_cls": kcs}

    def apply_batch(self, shapes) -> bool:
        """Set the batch class's stored team rule and chunk length together
        with every class's stored Gram unit shape.  Returns whether the batch
        class had an entry."""
        t = self.lookup(batch_class(shapes))
        merged = dict(t or {})
        merged.update(self.class_tuning())
        set_tuning(self.ctx, **merged)
        return t is not None

    # ---- measurement
    def _time(self, fn) -> float:
        import torch
        fn()  # warm-up (also grows the workspace)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(self.reps):
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            fn()
            e.record()
            e.synchronize()
            best = min(best, s.elapsed_time(e))
        return best

    def _record(self, key: str, tuning: dict, ms: float, trials):
        self.table[key] = {"tuning": tuning, "ms": ms, "trials": trials, "when": time.strftime("%Y-%m-%d %H:%M:%S")}

    def tune_dense(self, A, gram: str = "bf16x3", k: int = 8, power_iters: int = 20, branch: int = 0,
                   save: bool = True) -> dict:
        """Tune the Gram (tile, chunks) and then the power launch (workgroups)
        for A's class.  The power step is timed in fixed-iteration mode on the
        Gram of A, so every candidate does the same work."""
        import torch
        from . import tsvd_gram_dense, tsvd_power_gram
        m, n = A.shape
        right = (m > n) if branch == 1 else (m >= n)
        d, K = (n, m) if right else (m, n)
        key = dense_class(m, n, gram, branch)
        saved = get_tuning(self.ctx)
        trials = []
        side = "right" if right else "left"
        B = torch.empty((d, d), dtype=torch.float32, device=A.device)
        best_g, best_ms = None, float("inf")
        for tile, chunks in gram_candidates(gram, d, K, self.ctx.num_cu):
            set_tuning(self.ctx, gram_tile=tile, gram_chunks=chunks)
            ms = self._time(lambda: tsvd_gram_dense(self.ctx, A, gram=gram, side=side, B=B))
            trials.append({"gram_tile": tile, "gram_chunks": chunks, "gram_ms": ms})
            if ms < best_ms:
                best_g, best_ms = (tile, chunks), ms
        tile, chunks = best_g
        set_tuning(self.ctx, gram_tile=tile, gram_chunks=chunks)
        tsvd_gram_dense(self.ctx, A, gram=gram, side=side, B=B)
        gen = torch.Generator(device="cpu").manual_seed(1)
        v0 = torch.randn((k, d), generator=gen, dtype=torch.float64).to(A.device)
        Bw = torch.empty_like(B)
        best_p, best_pms = 0, float("inf")
        for g in power_candidates(d, self.ctx.num_cu):
            set_tuning(self.ctx, gram_tile=tile, gram_chunks=chunks, power_blocks=g)

            def run():
                Bw.copy_(B)
                tsvd_power_gram(self.ctx, Bw, k, 0.0, v0, fixed_iters=[power_iters] * k)
            ms = self._time(run)
            trials.append({"power_blocks": g, "power_ms": ms})
            if ms < best_pms:
                best_p, best_pms = g, ms
        tuning = {"gram_tile": tile, "gram_chunks": chunks, "power_blocks": best_p}
        self._record(key, tuning, best_ms + best_pms, trials)
        set_tuning(self.ctx, **saved)
        if save:
            self.save()
        return tuning

    def tune_batch(self, problems, save: bool = True) -> dict:
        """Tune team_kib and group_kchunk on a representative batch (the
        problem dicts of tsvd_dense_batched)."""
        from . import tsvd_dense_batched
        shapes = [tuple(p["A"].shape) for p in problems]
        key = batch_class(shapes)
        saved = get_tuning(self.ctx)
        trials = []
        best, best_ms = None, float("inf")
        for tk, kc in batch_candidates():
            set_tuning(self.ctx, team_kib=tk, group_kchunk=kc)
            ms = self._time(lambda: tsvd_dense_batched(self.ctx, problems))
            trials.append({"team_kib": tk, "group_kchunk": kc, "ms": ms})
            if ms < best_ms:
                best, best_ms = (tk, kc), ms
        tuning = {"team_kib": best[0], "group_kchunk": best[1]}
        self._record(key, tuning, best_ms, trials)
        set_tuning(self.ctx, **saved)
        if save:
            self.save()
        return tuning

    def tune_gram_classes(self, shapes, per_class: int = 16, seed: int = 7, save: bool = True) -> dict:
        """Tune the batched Gram's work unit (tile edge, chunk rows) per
        Gram-dimension class.  For every class that `shapes` (a list of (m, n))
        reaches, a batch of up to `per_class` of its shapes, with random A,
        one triplet and one fixed iteration (so that the Gram dominates the
        call), is timed under each candidate; the other classes keep their
        current entries.  Returns {class: (tile, chunk rows)}."""
        import torch
        from . import tsvd_dense_batched
        by_cls = {}
        for m, n in shapes:
            by_cls.setdefault(gram_class(min(m, n)), []).append((int(m), int(n)))
        saved = get_tuning(self.ctx)
        dev = torch.device("cuda", self.ctx.device)
        gen = torch.Generator(device=dev).manual_seed(int(seed))
        chosen = {}
        for c in sorted(by_cls):
            sub = by_cls[c][:per_class]
            probs = []
            for m, n in sub:
                A = torch.randn((m, n), generator=gen, dtype=torch.float32, device=dev)
                v0 = torch.randn((1, min(m, n)), generator=gen, dtype=torch.float64, device=dev)
                probs.append({"A": A, "k": 1, "eps": 0.0, "v0": v0, "fixed_iters": [1], "gram": "bf16x3"})
            K_max = max(max(m, n) for m, n in sub)
            trials = []
            best, best_ms = None, float("inf")
            for tile, kc in gram_unit_candidates(K_max):
                cur = self.class_tuning()
                cur["group_tile"][c], cur["group_kchunk_cls"][c] = tile, kc
                base = dict(saved)
                base.update(cur)
                set_tuning(self.ctx, **base)
                ms = self._time(lambda: tsvd_dense_batched(self.ctx, probs, raise_errors=True))
                trials.append({"group_tile": tile, "group_kchunk": kc, "ms": ms})
                if ms < best_ms:
                    best, best_ms = (tile, kc), ms
            self._record(gram_unit_key(c), {"group_tile": best[0], "group_kchunk": best[1]}, best_ms, trials)
            chosen[c] = best
        set_tuning(self.ctx, **saved)
        if save:
            self.save()
        return chosen
