"""Training data, training and evaluation of the learned cost model.

The learned model (a 40-128-128-128-1 ReLU network over the features the
scheduler computes for a (fusion group, configuration) pair) predicts the log
of the group's kernel time.  Its data are timings the library itself takes on
the device:

* ``collect``: for each pipeline, candidate groups (the analytical
  schedule's groups, every stage alone, and random connected convex groups of
  2..12 stages) are timed under several configurations each (the analytical
  model's pick and random draws from the search grid) through
  ``measure_groups``; every timing is appended to a JSON-lines database.
* ``train``: the network is trained on the device (the library's forward,
  backward and Adam kernels) on a split of the database by pipeline.
* ``evaluate``: for held-out pipelines, whole plans scheduled by the
  analytical model, by the learned model and by the autotuner are timed next
  to the unfused plan and to the best schedule assembled from the measured
  candidates (a dynamic program over measured group times), and both models'
  rankings are compared to the measurements (Kendall tau).

Command line: ``python -m paper_1909_07190_amd.learn collect|train|evaluate``.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import random
import re
import sys
import time

import numpy as np

from . import NUM_FEATURES, Mlp, from_spec, group_features, measure_groups

FUSABLE = ("stencil", "pointwise")


# ---------------------------------------------------------------- structure --

class Dag:
    """Stage structure of a plain-data pipeline spec, by library node id."""

    def __init__(self, spec, pipe):
        self.spec = spec
        self.pipe = pipe
        self.kind, self.level, self.prod = {}, {}, {}
        for inp in spec["inputs"]:
            i = pipe.names[inp["name"]]
            self.kind[i], self.level[i], self.prod[i] = "input", 0, []
        for st in spec["stages"]:
            i = pipe.names[st["name"]]
            srcs = [pipe.names[s] for s in st.get("srcs", [st.get("src")])]
            self.kind[i] = st["kind"]
            self.prod[i] = srcs
            lv = self.level[srcs[0]]
            self.level[i] = lv + 1 if st["kind"] == "down2" else lv - 1 if st["kind"] == "up2" else lv
        self.stages = sorted(i for i, k in self.kind.items() if k != "input")
        self.cons = {i: [] for i in self.kind}
        for i, ps in self.prod.items():
            for s in ps:
                self.cons[s].append(i)

    def fusable(self, i):
        return self.kind[i] in FUSABLE

    def _closure(self, start, nxt):
        seen, stack = set(), list(start)
        while stack:
            v = stack.pop()
            for u in nxt[v]:
                if u not in seen:
                    seen.add(u)
                    stack.append(u)
        return seen

    def convex(self, group):
        g = set(group)
        down = self._closure(g, self.cons) - g
        up = self._closure(g, self.prod) - g
        return not (down & up)

    def random_group(self, rng, size):
        seeds = [i for i in self.stages if self.fusable(i)]
        if not seeds:
            return None
        g = [rng.choice(seeds)]
        lvl = self.level[g[0]]
        for _ in range(4 * size):
            if len(g) >= size:
                break
            nb = sorted({u for v in g for u in self.prod[v] + self.cons[v]
                         if u not in g and self.kind[u] in FUSABLE and self.level[u] == lvl})
            if not nb:
                break
            u = rng.choice(nb)
            if self.convex(g + [u]):
                g.append(u)
        return sorted(g) if len(g) >= 2 else None


def all_groups(dag, max_size=10):
    """Every group of 2..max_size fusable stages of one level that is
    connected (a producer-consumer edge or a shared pipeline input between
    members) and convex: the fusion search's candidate set without
    resampling stages, enumerated exhaustively (each connected set once, by
    extending from its smallest stage with exclusive neighbourhoods)."""
    fus = [i for i in dag.stages if dag.fusable(i)]
    adj = {i: set() for i in fus}
    for i in fus:
        for u in dag.prod[i] + dag.cons[i]:
            if u in adj and dag.level[u] == dag.level[i]:
                adj[i].add(u)
                adj[u].add(i)
    for inp, kind in dag.kind.items():
        if kind != "input":
            continue
        readers = [i for i in dag.cons[inp] if i in adj]
        for a in readers:
            for b in readers:
                if a != b and dag.level[a] == dag.level[b]:
                    adj[a].add(b)
    out = []

    def extend(sub, ext, v):
        if len(sub) >= 2 and dag.convex(sorted(sub)):
            out.append(tuple(sorted(sub)))
        if len(sub) == max_size:
            return
        ext = set(ext)
        while ext:
            w = min(ext)
            ext.discard(w)
            near = set().union(*(adj[x] for x in sub)) | sub
            excl = {u for u in adj[w] if u > v and u not in near}
            extend(sub | {w}, ext | excl, v)

    for v in fus:
        extend({v}, {u for u in adj[v] if u > v}, v)
    return out


# tile configurations of the exhaustive search (every group under each)
EXHAUSTIVE_GRID = ("V=4 TX=1 SX=0 TY=16 PF=2", "V=4 TX=1 SX=0 TY=32 PF=2", "V=2 TX=1 SX=0 TY=16 PF=2",
                   "V=2 TX=2 SX=0 TY=16 PF=2", "V=4 TX=2 SX=0 TY=8 PF=2", "V=2 TX=1 SX=0 TY=32 PF=1",
                   "V=1 TX=4 SX=2 TY=16 PF=1", "V=4 TX=1 SX=1 TY=16 PF=2")


def exhaustive_schedule(dag, pipe, width, height, grid=EXHAUSTIVE_GRID, max_size=10, reps=20, log=None):
    """Measures every admissible group (and every stage alone) under every
    configuration of `grid`, then assembles the fastest schedule from the
    measurements (a dynamic program over down-closed stage sets); returns
    (total microseconds, schedule text, timings taken)."""
    groups = [(i,) for i in dag.stages if dag.fusable(i)] + all_groups(dag, max_size)
    texts = [_group_text(list(g), cfg) for g in groups for cfg in grid]
    times = []
    for c in range(0, len(texts), 96):  # in chunks, reporting progress
        times += measure_groups(pipe, texts[c:c + 96], width, height, reps=reps, tag="exhaustive")
        if log:
            log(f"exhaustive: {len(times)} of {len(texts)} candidates timed")
    rows = [{"group": t, "measured_us": us} for t, us in zip(texts, times) if math.isfinite(us)]
    res_us = {}
    for i in dag.stages:
        if not dag.fusable(i):
            t = measure_groups(pipe, [_group_text([i])], width, height, reps=reps)[0]
            res_us[i] = (t, _group_text([i]))
    total, text = best_measured_schedule(dag, rows, res_us)
    return total, text, len(texts)


def _group_text(nodes, cfg=""):
    return "nodes=" + ",".join(str(n) for n in nodes) + (" " + cfg if cfg else "")


def _parse_groups(describe_text):
    """(members plus decimated down2 stages, group text) per group of a plan
    description; the text keeps the group's decimated and expanded stages."""
    out = []
    for line in describe_text.strip().splitlines():
        toks = [t for t in line.split() if "=" in t and not t.startswith("batch_")]
        nodes = [int(x) for x in toks[0].split("=")[1].split(",")]
        for t in toks:
            if t.startswith("dec="):
                nodes += [int(x) for x in t[4:].split(",")]
        out.append((sorted(nodes), " ".join(toks)))
    return out


def _with_resampling(dag, group, rng):
    """The group with, for some members, their down2 written decimated and
    an up2 of that down2 folded in (the fusion search's cross-level groups),
    or the group unchanged."""
    out = list(group)
    for p in group:
        for d in dag.cons[p]:
            if dag.kind[d] != "down2" or rng.random() < 0.5:
                continue
            out.append(d)
            for u in dag.cons[d]:
                if dag.kind[u] == "up2" and rng.random() < 0.7:
                    out.append(u)
    return sorted(out)


# ------------------------------------------------------------------ collect --

def collect(specs, db, width=2048, height=2048, configs_per_group=4, random_groups=6,
            reps=20, seed=0, log=print, compile_only=False, picks_only=False):
    """Times candidate groups of every pipeline in `specs` (dict tag -> spec);
    appends to the database `db` (JSON lines).  The candidates of a pipeline
    depend only on (seed, tag), so `compile_only` can fill the code cache on a
    machine without a device ahead of the timing run.  With `picks_only`, only
    the groups of the analytical model's current plan, at its chosen
    configurations, are timed: the rows that correct the model where its own
    choices lead it (a refit on them is one round of learning from the
    model's mistakes)."""
    if not compile_only:
        os.environ["WT_MEASURE_DB"] = db
    n_total = 0
    for tag, spec in specs.items():
        # separate seeded streams: the random groups, and each group's
        # configurations, do not depend on the analytical schedule (so code
        # compiled ahead stays valid when the model changes)
        rng = random.Random(f"{seed}:{tag}:groups")
        t0 = time.time()
        pipe = from_spec(spec)
        dag = Dag(spec, pipe)
        texts = []
        groups = []
        for i in dag.stages:
            if picks_only:
                break
            groups.append(([i], 1 if dag.fusable(i) else 0))
            if not dag.fusable(i):
                texts.append(_group_text([i]))
        for _ in range(0 if picks_only else random_groups):
            g = dag.random_group(rng, rng.randint(2, 12))
            if g:
                groups.append((_with_resampling(dag, g, rng) if rng.random() < 0.5 else g, configs_per_group))
        plan = pipe.plan(width, height, mode="analytic", no_compile=True)
        for nodes, text in _parse_groups(plan.describe()):
            if not any(dag.fusable(n) for n in nodes):
                continue  # resampling kernels have no model features
            groups.append((nodes, 0 if picks_only else configs_per_group))
            texts.append(text)  # the analytical pick itself
        seen = set(texts)
        for nodes, k in groups:
            if k == 0:
                continue
            _, cfgs = group_features(pipe, nodes, width, height)
            cfgs = [c for c in cfgs if c]
            crng = random.Random(f"{seed}:{tag}:{','.join(map(str, nodes))}")
            for c in crng.sample(cfgs, min(k, len(cfgs))):
                if c not in seen:
                    seen.add(c)
                    texts.append(c)
        times = measure_groups(pipe, texts, width, height, reps=0 if compile_only else reps, tag=tag)
        n_total += len(texts)
        ok = sum(1 for t in times if math.isfinite(t))
        log(f"{'compile' if compile_only else 'collect'} {tag}: {len(spec['stages'])} stages, "
            f"{len(texts)} candidates ({ok} built), {time.time() - t0:.1f} s, {n_total} so far")
    return n_total


# -------------------------------------------------------------------- train --

def load_db(paths):
    rows = []
    for p in paths:
        with open(p) as f:
            for line in f:
                line = line.strip()
                if not line:
                    continue
                # non-finite model quantities (a configuration the model
                # deems infeasible) are written as null; older lines as inf
                line = re.sub(r"(?<=[\[ ,:])-?inf(?=[\],}])", "null", line)
                r = json.loads(line)
                feats = r.get("features") or []
                ok = (r["measured_us"] is not None and math.isfinite(r["measured_us"]) and r["measured_us"] > 0
                      and len(feats) == NUM_FEATURES and all(v is not None and math.isfinite(v) for v in feats)
                      and r.get("pred_us") is not None and all(t is not None for t in r.get("terms", [])))
                if ok:
                    rows.append(r)
    return rows


def split_by_holdout(rows, path):
    """(train tags, test tags) with the test tags read from `path` (one per
    line), so a split survives the database growing."""
    with open(path) as f:
        te = {ln.strip() for ln in f if ln.strip()}
    tags = {r["pipeline"] for r in rows}
    return tags - te, tags & te


def split_tags(rows, test_fraction=0.2, seed=0):
    tags = sorted({r["pipeline"] for r in rows})
    rng = random.Random(seed)
    rng.shuffle(tags)
    ntest = max(1, int(round(len(tags) * test_fraction))) if len(tags) > 1 else 0
    return set(tags[ntest:]), set(tags[:ntest])


def train(rows, model_path, log=print):
    """Trains the cost network on `rows` through the library's
    wt_model_train (the rows are written to a JSON-lines file beside the
    model, which the library parses, standardises and trains on)."""
    from . import model_rows, model_train
    db = model_path + ".train.jsonl"
    with open(db, "w") as f:
        for r in rows:
            f.write(json.dumps(r) + "\n")
    assert model_rows(db) == len(rows)
    t0 = time.time()
    model_train(db, model_path)
    os.remove(db)
    log(f"train: {len(rows)} rows, {time.time() - t0:.1f} s")
    return Mlp.load(model_path)


def kendall_tau(a, b):
    n, s = len(a), 0
    cnt = 0
    for i in range(n):
        for j in range(i + 1, n):
            d = (a[i] - a[j]) * (b[i] - b[j])
            if d > 0:
                s += 1
            elif d < 0:
                s -= 1
            cnt += 1
    return s / cnt if cnt else float("nan")


def ranking_report(rows, net, fit=None):
    """Per group (same pipeline and node set, two or more configurations):
    Kendall tau of the analytical predicted time (and of its calibrated form
    under `fit`, when given), Algorithm 2's score and the network's
    prediction against the measurements, and the regret of each model's top
    pick (its measured time over the best measured)."""
    by = {}
    for r in rows:
        key = (r["pipeline"], r["group"].split()[0])
        by.setdefault(key, []).append(r)
    names = ["analytic_pred"] + (["analytic_calibrated"] if fit else []) + ["alg2_score", "mlp"]
    taus = {n: [] for n in names}
    regret = {n: [] for n in names}
    for rs in by.values():
        if len(rs) < 2:
            continue
        meas = [r["measured_us"] for r in rs]
        preds = {"analytic_pred": [r["pred_us"] for r in rs], "alg2_score": [r["score"] for r in rs],
                 "mlp": list(np.exp(net.predict(np.array([r["features"] for r in rs], np.float32))))}
        if fit:
            preds["analytic_calibrated"] = [calibrated(fit, r) for r in rs]
        for name in names:
            pred = preds[name]
            taus[name].append(kendall_tau(pred, meas))
            regret[name].append(meas[int(np.argmin(pred))] / min(meas))
    out = {}
    for name in taus:
        t = [v for v in taus[name] if math.isfinite(v)]
        out[name] = {"groups": len(t), "kendall_tau_mean": float(np.mean(t)) if t else None,
                     "top1_regret_geomean": float(np.exp(np.mean(np.log(regret[name])))) if regret[name] else None}
    return out


# ------------------------------------------------------- analytical refit --

def fit_analytic(rows, weights=None):
    """Refits the analytical model on gfx950 measurements: least squares of
    log(measured time) on an intercept, log(the roofline-style predicted
    time) and Algorithm 2's seven terms, with non-negative coefficients on
    the terms (they are penalties) and on log(predicted time).  Returns
    {"c0", "c1", "w": [7]}; the model's calibrated time is
    exp(c0 + c1 log(pred_us) + sum_k w_k term_k).  `weights` (one per row)
    weight the squared residuals."""
    from scipy.optimize import lsq_linear

    if weights is None:
        weights = [1.0] * len(rows)
    keep = [i for i, r in enumerate(rows) if math.isfinite(r.get("pred_us", float("inf"))) and r["pred_us"] > 0]
    rows = [rows[i] for i in keep]
    sw = np.sqrt(np.array([weights[i] for i in keep], np.float64))
    a = np.array([[1.0, math.log(r["pred_us"])] + list(r["terms"]) for r in rows]) * sw[:, None]
    b = np.log(np.array([r["measured_us"] for r in rows])) * sw
    lo = [-np.inf] + [0.0] * 8
    res = lsq_linear(a, b, bounds=(lo, [np.inf] * 9))
    x = res.x
    return {"c0": float(x[0]), "c1": float(x[1]), "w": [float(v) for v in x[2:]], "rows": len(rows)}


def calibrated(fit, r):
    return math.exp(fit["c0"] + fit["c1"] * math.log(r["pred_us"]) +
                    sum(w * t for w, t in zip(fit["w"], r["terms"])))


def analytic_report(rows, fit):
    """Top-1 regret (geomean over groups) and Kendall tau of the calibrated
    time, and the log-space correlation with the measurements."""
    by = {}
    for r in rows:
        by.setdefault((r["pipeline"], r["group"].split()[0]), []).append(r)
    taus, reg = [], []
    for rs in by.values():
        if len(rs) < 2:
            continue
        meas = [r["measured_us"] for r in rs]
        pred = [calibrated(fit, r) for r in rs]
        taus.append(kendall_tau(pred, meas))
        reg.append(meas[int(np.argmin(pred))] / min(meas))
    lm = np.log([r["measured_us"] for r in rows])
    lp = np.log([calibrated(fit, r) for r in rows])
    return {"groups": len(reg), "kendall_tau_mean": float(np.nanmean(taus)) if taus else None,
            "top1_regret_geomean": float(np.exp(np.mean(np.log(reg)))) if reg else None,
            "log_corr": float(np.corrcoef(lm, lp)[0, 1]) if len(rows) > 2 else None,
            "median_abs_log_err": float(np.median(np.abs(lm - lp)))}


# ----------------------------------------------------------------- evaluate --

def _time_plan(torch, plan, ins, outs, reps=20):
    for _ in range(3):
        plan.run(ins, outs)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.run(ins, outs)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e3 / reps)
    return best


def best_measured_schedule(dag, rows, resample_us):
    """Minimum-total-time partition of the stages into measured candidate
    groups (each at its best measured configuration), by a dynamic program over
    down-closed stage sets; returns (total microseconds, schedule text)."""
    best = {}
    for r in rows:
        nodes = tuple(int(x) for x in r["group"].split()[0].split("=")[1].split(","))
        if nodes not in best or r["measured_us"] < best[nodes][0]:
            best[nodes] = (r["measured_us"], r["group"])
    for i, (us, text) in resample_us.items():
        best[(i,)] = (us, text)
    stages = dag.stages
    bit = {s: 1 << k for k, s in enumerate(stages)}
    full = (1 << len(stages)) - 1
    cand = []
    for nodes, (us, text) in best.items():
        m = 0
        for n in nodes:
            m |= bit[n]
        need = 0
        for n in nodes:
            for p in dag.prod[n]:
                if p in bit and not (m & bit[p]):
                    need |= bit[p]
        cand.append((m, need, us, text))
    memo = {}

    def solve(S):
        if S == full:
            return 0.0, []
        if S in memo:
            return memo[S]
        res = (float("inf"), [])
        for m, need, us, text in cand:
            if m & S or (need & ~S):
                continue
            t, rest = solve(S | m)
            if us + t < res[0]:
                res = (us + t, [text] + rest)
        memo[S] = res
        return res

    sys.setrecursionlimit(10000)
    t, texts = solve(0)
    return t, ";".join(texts)


ALL_MODES = ("unfused", "analytic", "mlp", "autotune", "mlp_autotune", "best_measured", "exhaustive")
# modes that use the learned model (excluded from the reference it is judged by)
LEARNED_MODES = ("mlp", "mlp_autotune")


def evaluate(specs, rows, model_path, width=2048, height=2048, autotune_topk=4, log=print, out_path=None,
             modes=ALL_MODES, exhaustive_max_stages=10):
    import torch

    dev = torch.device("cuda:0")
    results = []
    for tag, spec in specs.items():
        pipe = from_spec(spec)
        dag = Dag(spec, pipe)
        gen = torch.Generator(device=dev)
        gen.manual_seed(len(results) + 1)
        ins = [torch.rand((1, height, width), device=dev, generator=gen) for _ in spec["inputs"]]
        outs = []
        for o in spec["outputs"]:
            lv = dag.level[pipe.names[o]]
            w, h = width, height
            for _ in range(lv):
                w, h = (w + 1) // 2, (h + 1) // 2
            outs.append(torch.empty((1, h, w), device=dev))
        res = {"pipeline": tag, "stages": len(spec["stages"])}
        make = {
            "unfused": lambda: pipe.plan(width, height, mode="unfused"),
            "analytic": lambda: pipe.plan(width, height, mode="analytic"),
            "mlp": lambda: pipe.plan(width, height, mode="mlp", model_path=model_path),
            "autotune": lambda: pipe.plan(width, height, mode="autotune", autotune_topk=autotune_topk),
            "mlp_autotune": lambda: pipe.plan(width, height, mode="autotune", autotune_topk=autotune_topk,
                                              model_path=model_path),
        }
        plans = {}
        for m in modes:
            if m in make:
                log(f"{tag}: planning {m}")
                plans[m] = make[m]()
        drows = [r for r in rows if r["pipeline"] == tag]
        if drows and "best_measured" in modes:
            res_us = {}
            for i in dag.stages:
                if not dag.fusable(i):
                    t = measure_groups(pipe, [_group_text([i])], width, height)[0]
                    res_us[i] = (t, _group_text([i]))
            t_sum, text = best_measured_schedule(dag, drows, res_us)
            if math.isfinite(t_sum):
                plans["best_measured"] = pipe.plan(width, height, mode="fixed", fixed=text)
                res["best_measured_sum_us"] = t_sum
        if "exhaustive" in modes and len(spec["stages"]) <= exhaustive_max_stages:
            t_sum, text, n = exhaustive_schedule(dag, pipe, width, height, log=log)
            if math.isfinite(t_sum):
                plans["exhaustive"] = pipe.plan(width, height, mode="fixed", fixed=text)
                res["exhaustive_sum_us"] = t_sum
                res["exhaustive_timings"] = n
        for name, plan in plans.items():
            res[name + "_us"] = _time_plan(torch, plan, ins, outs)
            res[name + "_groups"] = plan.num_groups
        timed = {k[:-3]: v for k, v in res.items() if k.endswith("_us") and not k.endswith("sum_us")}
        res["best_us"] = min(timed.values())
        # the reference the learned model is judged by: the fastest plan no
        # learned mode produced (the exhaustive search where it ran)
        res["ref_us"] = min(v for k, v in timed.items() if k not in LEARNED_MODES)
        results.append(res)
        log(json.dumps(res))
        if out_path:  # one line per pipeline as it completes
            with open(out_path, "a") as f:
                f.write(json.dumps(res) + "\n")
    return results


def summarize(results):
    def gm(xs):
        xs = [x for x in xs if x > 0 and math.isfinite(x)]
        return float(np.exp(np.mean(np.log(xs)))) if xs else None

    out = {"pipelines": len(results)}
    for m in ("analytic", "mlp", "autotune", "mlp_autotune", "best_measured", "exhaustive", "unfused"):
        r = [x[m + "_us"] / x["best_us"] for x in results if m + "_us" in x]
        if r:
            out[m] = {"geomean_over_best": gm(r), "within_10pct": float(np.mean([v <= 1.10 for v in r])),
                      "pipelines": len(r)}
            ref = [x[m + "_us"] / x["ref_us"] for x in results if m + "_us" in x and "ref_us" in x]
            if ref:
                out[m]["geomean_over_reference"] = gm(ref)
                out[m]["within_10pct_of_reference"] = float(np.mean([v <= 1.10 for v in ref]))
    ex = [x for x in results if "exhaustive_us" in x]
    if ex:
        out["exhaustive_pipelines"] = len(ex)
        for m in ("mlp", "mlp_autotune", "analytic"):
            r = [x[m + "_us"] / x["exhaustive_us"] for x in ex if m + "_us" in x]
            if r:
                out[m + "_over_exhaustive"] = {"geomean": gm(r), "within_10pct": float(np.mean([v <= 1.10 for v in r]))}
    out["mlp_gain_over_analytic"] = gm([x["analytic_us"] / x["mlp_us"] for x in results
                                         if "analytic_us" in x and "mlp_us" in x])
    out["mlp_speedup_over_unfused"] = gm([x["unfused_us"] / x["mlp_us"] for x in results
                                           if "unfused_us" in x and "mlp_us" in x])
    return out


# ---------------------------------------------------------------------- cli --

def _seeds(text):
    out = []
    for part in text.split(","):
        if "-" in part:
            a, b = part.split("-")
            out.extend(range(int(a), int(b) + 1))
        else:
            out.append(int(part))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1909_07190_amd.learn")
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect", help="time candidate groups of random pipelines")
    c.add_argument("--seeds", required=True, help="random pipeline seeds, e.g. 0-99")
    c.add_argument("--db", required=True)
    c.add_argument("--configs", type=int, default=4)
    c.add_argument("--random-groups", type=int, default=6)
    c.add_argument("--size", type=int, default=2048)
    c.add_argument("--compile-only", action="store_true",
                   help="only compile the candidates into $WT_CACHE_DIR (no device needed)")
    c.add_argument("--picks-only", action="store_true",
                   help="time only the analytical model's current picks")
    t = sub.add_parser("train", help="train the network on the device")
    t.add_argument("--db", required=True, nargs="+")
    t.add_argument("--holdout", help="file of held-out pipeline tags (default: a seeded fifth)")
    t.add_argument("--model", required=True)
    t.add_argument("--report", help="write the ranking report (JSON) here")
    f = sub.add_parser("fit-analytic", help="refit the analytical model's coefficients")
    f.add_argument("--db", required=True, nargs="+")
    f.add_argument("--holdout", help="file of held-out pipeline tags (default: a seeded fifth)")
    f.add_argument("--out", help="write the fit and its report (JSON) here")
    f.add_argument("--picks-db", nargs="+", help="rows of the model's own picks, from collect --picks-only")
    f.add_argument("--picks-weight", type=float, default=5.0, help="weight of each picks row in the fit")
    e = sub.add_parser("evaluate", help="compare whole-plan schedules on held-out pipelines")
    e.add_argument("--db", nargs="+", help="measurement database (its held-out pipelines are evaluated)")
    e.add_argument("--seeds", help="evaluate these random pipelines instead (no database needed)")
    e.add_argument("--stages", default="8-24", help="stage-count range of the --seeds pipelines, e.g. 6-9")
    e.add_argument("--holdout", help="file of held-out pipeline tags (default: a seeded fifth)")
    e.add_argument("--model", required=True)
    e.add_argument("--max-pipelines", type=int, default=0)
    e.add_argument("--skip", type=int, default=0, help="skip the first held-out pipelines")
    e.add_argument("--size", type=int, default=2048)
    e.add_argument("--out", help="append per-pipeline JSON lines here")
    e.add_argument("--modes", help="comma-separated subset of " + ",".join(ALL_MODES))
    sm = sub.add_parser("summarize", help="summarise per-pipeline evaluation lines")
    sm.add_argument("--results", required=True, nargs="+")
    a = ap.parse_args(argv)

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from synth import dags

    def log(m):
        print(m, flush=True)

    if a.cmd == "collect":
        specs = {f"dag{s}": dags.random_dag(s) for s in _seeds(a.seeds)}
        collect(specs, a.db, a.size, a.size, a.configs, a.random_groups, log=log,
                compile_only=a.compile_only, picks_only=a.picks_only)
    elif a.cmd == "train":
        rows = load_db(a.db)
        tr, te = split_by_holdout(rows, a.holdout) if a.holdout else split_tags(rows)
        train_rows = [r for r in rows if r["pipeline"] in tr]
        net = train(train_rows, a.model, log=log)
        fit = fit_analytic(train_rows)
        rep = {"train_pipelines": len(tr), "test_pipelines": len(te), "train_rows": len(train_rows),
               "test_rows": len(rows) - len(train_rows), "analytic_fit": fit,
               "train": ranking_report(train_rows, net, fit),
               "test": ranking_report([r for r in rows if r["pipeline"] in te], net, fit)}
        log(json.dumps(rep))
        if a.report:
            with open(a.report, "w") as f:
                json.dump(rep, f, indent=1)
    elif a.cmd == "fit-analytic":
        rows = load_db(a.db)
        tr, te = split_by_holdout(rows, a.holdout) if a.holdout else split_tags(rows)
        train_rows = [r for r in rows if r["pipeline"] in tr]
        test_rows = [r for r in rows if r["pipeline"] in te]
        # the model's own picks (collect --picks-only) on training pipelines
        picks = [r for r in load_db(a.picks_db) if r["pipeline"] in tr] if a.picks_db else []
        fit = fit_analytic(train_rows + picks, [1.0] * len(train_rows) + [a.picks_weight] * len(picks))
        fit["picks_rows"] = len(picks)
        rep = {"fit": fit, "train": analytic_report(train_rows, fit), "test": analytic_report(test_rows, fit)}
        log(json.dumps(rep))
        if a.out:
            with open(a.out, "w") as fh:
                json.dump(rep, fh, indent=1)
    elif a.cmd == "summarize":
        res = []
        for path in a.results:
            with open(path) as f:
                res.extend(json.loads(line) for line in f if line.strip())
        log(json.dumps(summarize(res)))
    elif a.cmd == "evaluate":
        if a.seeds:
            # pipelines no campaign measured, so none the network trained on
            rows = []
            lo, hi = (int(x) for x in a.stages.split("-"))
            specs = {f"dag{s}": dags.random_dag(s, lo=lo, hi=hi) for s in _seeds(a.seeds)}
        else:
            if not a.db:
                ap.error("evaluate needs --db or --seeds")
            rows = load_db(a.db)
            _, te = split_by_holdout(rows, a.holdout) if a.holdout else split_tags(rows)
            tags = sorted(te, key=lambda s: int(s[3:]) if s[3:].isdigit() else s)
            tags = tags[a.skip:]
            if a.max_pipelines:
                tags = tags[:a.max_pipelines]
            specs = {tg: dags.random_dag(int(tg[3:])) for tg in tags}
        modes = tuple(a.modes.split(",")) if a.modes else ALL_MODES
        res = evaluate(specs, rows, a.model, a.size, a.size, log=log, out_path=a.out, modes=modes)
        log(json.dumps(summarize(res)))


if __name__ == "__main__":
    main()
