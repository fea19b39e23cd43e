"""Serving: binding of the lola_server calls and a driver for the mixed
workload (Poisson arrivals of N=16384 MNIST-shaped and N=4096 dense-64
queries, several resident client key sets per ring size).

The driver submits requests at their arrival times, steps the server
(continuous batching across requests and ring sizes), measures each request's
latency from arrival to observed completion, checks every served result word
for word against the reference words of its (client, input set) -- that
pair evaluated alone once -- and a sample against the same request evaluated
alone again afterwards, and replays
the same arrival trace through the one-request-at-a-time GPU path for
comparison.  Argument marshalling and bookkeeping only: all homomorphic work
runs in the library.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np
import torch

from . import lola, networks
from . import workloads as wl


def _sig():
    L = lola._plan_sig()
    if getattr(L, "_srv_sig", False):
        return L
    vp, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "lola_server_create": [ctypes.c_size_t, ctypes.POINTER(vp)],
        "lola_server_add_model": [vp, vp, vp, u32, ctypes.POINTER(u32)],
        "lola_server_model_info": [vp, u32, ctypes.POINTER(u32), ctypes.POINTER(u64), ctypes.POINTER(u64),
                                   ctypes.POINTER(u64)],
        "lola_server_submit": [vp, u32, ctypes.POINTER(lola.Request), u64],
        "lola_server_set_solo_plan": [vp, u32, vp],
        "lola_server_submit_ex": [vp, u32, ctypes.POINTER(lola.Request), ctypes.POINTER(vp), u64],
        "lola_server_step": [vp, ctypes.POINTER(u32)],
        "lola_server_poll": [vp, ctypes.POINTER(u64), u32, ctypes.POINTER(u32)],
        "lola_server_poll_ex": [vp, ctypes.POINTER(u64), ctypes.POINTER(u32), u32, ctypes.POINTER(u32)],
        "lola_server_destroy": [vp],
    }
    for n, a in sig.items():
        f = getattr(L, n)
        f.argtypes = a
        f.restype = ctypes.c_int32
    L.lola_server_destroy.restype = None
    L._srv_sig = True
    return L


def _request_struct(r, keep):
    gk = (ctypes.c_void_p * max(len(r["gks"]), 1))(*[t.data_ptr() for t in r["gks"]])
    ins = (ctypes.c_void_p * len(r["inputs"]))(*[t.data_ptr() for t in r["inputs"]])
    outs = (ctypes.c_void_p * len(r["outputs"]))(*[t.data_ptr() for t in r["outputs"]])
    keep += [gk, ins, outs]
    return lola.Request(r["rlk"].data_ptr() if r.get("rlk") is not None else None,
                        ctypes.cast(gk, ctypes.POINTER(ctypes.c_void_p)),
                        ctypes.cast(ins, ctypes.POINTER(ctypes.c_void_p)),
                        ctypes.cast(outs, ctypes.POINTER(ctypes.c_void_p)))


class Server:
    def __init__(self, hbm_budget_bytes: int):
        L = _sig()
        h = ctypes.c_void_p()
        lola._check(L.lola_server_create(hbm_budget_bytes, ctypes.byref(h)))
        self.h = h

    def add_model(self, ctx, plan, max_inflight: int) -> int:
        mid = ctypes.c_uint32()
        lola._check(_sig().lola_server_add_model(self.h, ctx.h, plan.h, max_inflight, ctypes.byref(mid)))
        return mid.value

    def model_info(self, mid: int):
        s, f, sc, j = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        lola._check(_sig().lola_server_model_info(self.h, mid, ctypes.byref(s), ctypes.byref(f), ctypes.byref(sc),
                                                  ctypes.byref(j)))
        return dict(slots=s.value, footprint_bytes=f.value, scratch_bytes=sc.value, launched_jobs=j.value)

    def set_solo_plan(self, mid: int, plan) -> None:
        lola._check(_sig().lola_server_set_solo_plan(self.h, mid, plan.h))

    def submit(self, mid: int, req: dict, tag: int) -> None:
        """req may carry gks_solo, the solo plan's Galois keys."""
        keep = []
        rs = _request_struct(req, keep)
        solo = None
        if req.get("gks_solo") is not None:
            arr = (ctypes.c_void_p * max(len(req["gks_solo"]), 1))(*[t.data_ptr() for t in req["gks_solo"]])
            keep.append(arr)
            solo = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
        lola._check(_sig().lola_server_submit_ex(self.h, mid, ctypes.byref(rs), solo, tag))

    def step(self) -> int:
        n = ctypes.c_uint32()
        lola._check(_sig().lola_server_step(self.h, ctypes.byref(n)))
        return n.value

    def poll(self, cap: int = 4096):
        """Tags completed since the last poll; self.forms[tag] = 1 if the solo
        plan served it, else 0."""
        tags = (ctypes.c_uint64 * cap)()
        forms = (ctypes.c_uint32 * cap)()
        n = ctypes.c_uint32()
        lola._check(_sig().lola_server_poll_ex(self.h, tags, forms, cap, ctypes.byref(n)))
        if not hasattr(self, "forms"):
            self.forms = {}
        for i in range(n.value):
            self.forms[int(tags[i])] = int(forms[i])
        return [int(tags[i]) for i in range(n.value)]

    def close(self):
        if getattr(self, "h", None):
            _sig().lola_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


class ModelSetup:
    """A ring size's context, loaded plan (and solo plan: the network compiled
    for the latency objective, where that differs), client key sets with the
    Galois keys of both plans, pre-encrypted input sets and a pool of output
    buffers."""

    def __init__(self, kind: str, clients: int, inputs_per_client: int, out_pool: int,
                 mnist_params: str = "mnist_n16384_k2"):
        self.kind = kind
        if kind == "mnist":
            self.p = wl.PARAMS[mnist_params]
            self.w = wl.mnist_weights()
            layers = networks.mnist_layers(self.w)
        else:
            self.p = wl.PARAMS["n4096_3q"]
            _, self.W = wl.dense64_inputs()
            layers = networks.dense64_layers(self.W)
        self.ctx = lola.Context(self.p)
        self.plan = lola.Plan(self.p, layers)
        self.plan.load(self.ctx)
        solo = lola.Plan(self.p, layers, objective=lola.OBJECTIVE_LATENCY)
        if (solo.info["recipe"], solo.info["sums"]) != (self.plan.info["recipe"], self.plan.info["sums"]):
            self.solo_plan = solo
            self.solo_plan.load(self.ctx)
        else:
            solo.close()
            self.solo_plan = None
        gal = self.plan.galois()
        gal_solo = self.solo_plan.galois() if self.solo_plan is not None else []
        imap = self.plan.input_map()
        self.keys, self.inputs, self.values = [], [], []
        base = wl.workload_seed(4) * 31 + (1 if kind == "mnist" else 2)
        self.key_seeds, self.enc_seeds = [], []
        for c in range(clients):
            ks = base + 1009 * c
            self.key_seeds.append(ks)
            self.enc_seeds.append([ks + 7 * k + 3 for k in range(inputs_per_client)])
            sk = self.ctx.keygen_secret(ks)
            pk = self.ctx.keygen_public(ks, sk)
            gk = {g: self.ctx.keygen_switch(ks, sk, g) for g in sorted(set(gal) | set(gal_solo))}
            self.keys.append(dict(sk=sk, rlk=self.ctx.keygen_switch(ks, sk, 0), gks=[gk[g] for g in gal],
                                  gks_solo=[gk[g] for g in gal_solo] if self.solo_plan is not None else None))
            sets, vals = [], []
            for k in range(inputs_per_client):
                g = wl.rng(base + c, 100 + k)
                if kind == "mnist":
                    v = networks.mnist_input_values(g.integers(0, 256, size=(28, 28)))
                else:
                    v = g.integers(-128, 128, size=64)
                msgs = networks.pack_inputs(imap, v)
                sets.append([self.ctx.encrypt(pk, self.ctx.encode(m), ks + 7 * k + 3, i) for i, m in enumerate(msgs)])
                vals.append(v)
            self.inputs.append(sets)
            self.values.append(vals)
        self._refs = {}
        n_out = self.plan.info["n_outputs"]
        self.free_outputs = [[self.ctx.empty_ct() for _ in range(n_out)] for _ in range(out_pool)]

    def request(self, client: int, which: int, outputs):
        k = self.keys[client]
        return dict(rlk=k["rlk"], gks=k["gks"], gks_solo=k["gks_solo"], inputs=self.inputs[client][which],
                    outputs=outputs)

    def plan_of(self, form: int):
        """The plan that serves form 0 (the model's plan) or 1 (the solo plan)."""
        return self.solo_plan if form == 1 else self.plan

    def evaluate_alone(self, client: int, which: int, outputs, form: int = 0) -> None:
        """(client, input set) evaluated alone under the plan of the form."""
        req = self.request(client, which, outputs)
        if form == 1:
            req = dict(req, gks=req["gks_solo"])
        self.plan_of(form).evaluate(self.ctx, [req])

    def reference(self, client: int, which: int, form: int = 0):
        """The output words of (client, input set) evaluated alone under the
        plan of the form, computed once and kept."""
        key = (client, which, form)
        if key not in self._refs:
            outs = [self.ctx.empty_ct() for _ in range(self.plan.info["n_outputs"])]
            self.evaluate_alone(client, which, outs, form)
            torch.cuda.synchronize()
            self._refs[key] = outs
        return self._refs[key]


def run_serving(n_req: int = 2000, rate: float = 200.0, p_large: float = 0.7, clients: int = 8,
                max_inflight: int = 64, hbm_budget_gb: float = 96.0, check_every: int = 50,
                baseline: bool = True, seed: int | None = None, check_all: bool = True,
                keep_models: bool = False, mnist_params: str = "mnist_n16384_k2") -> dict:
    assert torch.cuda.is_available()
    arrivals, kinds = wl.serving_arrivals(n_req, rate, p_large, seed)
    g = wl.rng(wl.workload_seed(4) if seed is None else seed, 9)
    client_of = g.integers(0, clients, size=n_req)
    input_of = g.integers(0, 2, size=n_req)
    models = {"mnist": ModelSetup("mnist", clients, 2, max_inflight + 16, mnist_params),
              "dense64": ModelSetup("dense64", clients, 2, max_inflight + 16)}
    torch.cuda.synchronize()
    srv = Server(int(hbm_budget_gb * (1 << 30)))
    mids = {k: srv.add_model(m.ctx, m.plan, max_inflight) for k, m in models.items()}
    for k, m in models.items():
        if m.solo_plan is not None:
            srv.set_solo_plan(mids[k], m.solo_plan)
    kind_name = lambda k: "mnist" if k == 1 else "dense64"  # noqa: E731
    out_of, latency, served_copy, kept = {}, np.zeros(n_req), {}, {}
    pending = []          # arrived but waiting for an output buffer
    copying = []          # (event, model, buffers): returned to the pool once their copies are done
    nxt, done = 0, 0
    t0 = time.perf_counter()
    while done < n_req:
        while copying and copying[0][0].query():
            _, m, bufs = copying.pop(0)
            m.free_outputs.append(bufs)
        now = time.perf_counter() - t0
        while nxt < n_req and arrivals[nxt] <= now:
            pending.append(nxt)
            nxt += 1
        still = []
        for r in pending:
            m = models[kind_name(kinds[r])]
            if not m.free_outputs:
                still.append(r)
                continue
            outs = m.free_outputs.pop()
            out_of[r] = outs
            srv.submit(mids[m.kind], m.request(int(client_of[r]), int(input_of[r]), outs), r)
        pending = still
        inflight = srv.step()
        for tag in srv.poll():
            latency[tag] = time.perf_counter() - t0 - arrivals[tag]
            m = models[kind_name(kinds[tag])]
            bufs = out_of.pop(tag)
            copied = False
            if tag % check_every == 0:
                served_copy[tag] = [o.clone() for o in bufs]
                copied = True
            if check_all:
                kept[tag] = [o.clone() for o in bufs]
                copied = True
            if copied:
                # the copies run on torch's stream, which does not order with
                # the server's streams: the buffers go back to the pool (and
                # to a later request) only once the copies have completed
                ev = torch.cuda.Event()
                ev.record()
                copying.append((ev, m, bufs))
            else:
                m.free_outputs.append(bufs)
            done += 1
        if inflight == 0 and not pending and not copying and nxt < n_req:
            time.sleep(max(0.0, min(0.002, arrivals[nxt] - (time.perf_counter() - t0))))
    wall = time.perf_counter() - t0
    torch.cuda.synchronize()
    # served results equal the request evaluated alone, word for word
    # (under the plan that served it: the model's, or its solo plan)
    forms = srv.forms if hasattr(srv, "forms") else {}
    mismatches = 0
    for tag, outs in served_copy.items():
        m = models[kind_name(kinds[tag])]
        alone = [m.ctx.empty_ct() for _ in outs]
        m.evaluate_alone(int(client_of[tag]), int(input_of[tag]), alone, forms.get(tag, 0))
        torch.cuda.synchronize()
        mismatches += sum(0 if torch.equal(a, b) else 1 for a, b in zip(alone, outs))
    # every served result equals its (client, input set)'s reference words
    ref_mismatches = 0
    for tag, outs in kept.items():
        ref = models[kind_name(kinds[tag])].reference(int(client_of[tag]), int(input_of[tag]), forms.get(tag, 0))
        ref_mismatches += sum(0 if torch.equal(a, b) else 1 for a, b in zip(ref, outs))
    kept.clear()
    res = {
        "requests": n_req, "rate_per_s": rate, "wall_s": round(wall, 3), "mnist_params": mnist_params,
        "inferences_per_s": round(n_req / wall, 2),
        "p50_ms": round(float(np.percentile(latency, 50)) * 1e3, 2),
        "p99_ms": round(float(np.percentile(latency, 99)) * 1e3, 2),
        "by_model": {},
        "checked_alone_vs_mixed": len(served_copy), "mismatches": mismatches,
        "checked_vs_reference": n_req if check_all else 0, "reference_mismatches": ref_mismatches,
        "references": {k: len(m._refs) for k, m in models.items()},
        "served_by_solo_plan": {k: sum(1 for t, f in forms.items() if f == 1 and kind_name(kinds[t]) == k)
                                for k in models},
        "slots": {k: srv.model_info(v)["slots"] for k, v in mids.items()},
        "scratch_bytes": {k: srv.model_info(v)["scratch_bytes"] for k, v in mids.items()},
    }
    for k in (1, 0):
        sel = kinds == k
        if sel.any():
            res["by_model"][kind_name(k)] = {"n": int(sel.sum()),
                                             "p50_ms": round(float(np.percentile(latency[sel], 50)) * 1e3, 2),
                                             "p99_ms": round(float(np.percentile(latency[sel], 99)) * 1e3, 2)}
    srv.close()
    if baseline:
        res["one_at_a_time"] = one_at_a_time(models, arrivals, kinds, client_of, input_of)
    if keep_models:
        res["_models"] = models
    return res


def one_at_a_time(models, arrivals, kinds, client_of, input_of) -> dict:
    """The same arrival trace served by evaluating one request at a time, in
    arrival order, on the GPU (each request waits for the previous one), each
    under the model's plan for a request alone (its solo plan where it has
    one)."""
    n = len(arrivals)
    outs = {k: [m.ctx.empty_ct() for _ in range(m.plan.info["n_outputs"])] for k, m in models.items()}
    lat = np.zeros(n)
    t0 = time.perf_counter()
    for r in range(n):
        now = time.perf_counter() - t0
        if now < arrivals[r]:
            time.sleep(arrivals[r] - now)
        k = "mnist" if kinds[r] == 1 else "dense64"
        m = models[k]
        m.evaluate_alone(int(client_of[r]), int(input_of[r]), outs[k], 1 if m.solo_plan is not None else 0)
        torch.cuda.synchronize()
        lat[r] = time.perf_counter() - t0 - arrivals[r]
    wall = time.perf_counter() - t0
    return {"inferences_per_s": round(n / wall, 2), "wall_s": round(wall, 3),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2)}


if __name__ == "__main__":
    import json
    import sys
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 2000
    print(json.dumps(run_serving(n_req=n)), flush=True)
