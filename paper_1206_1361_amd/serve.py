"""Serving load: Poisson arrivals of mixed solve requests against gp_server.

    python -m paper_1206_1361_amd.serve [--rate 50] [--seconds 60] [--dtype c64]
        [--budget-gib 2] [--slots 96] [--check-every 10] [--verify 8] [--real-states]

Requests arrive as a seeded Poisson process.  70% are imaginary-time ground
states (Gaussian start of the request's own trap, stopped when mu moves by
less than 1e-8 between checks, at most 20000 steps), 30% are real-time
interaction quenches (the same Gaussian -- the g = 0 ground state --
evolved 2000 steps at the request's g).  Grids are drawn uniformly from
64^3, 96^3, 128^3 and 160x128x96, traps uniformly from [0.5, 3] per axis, g
uniformly from [1, 500]; dx = 0.2, dt = 0.1 dx^2 (imaginary) or 0.005 dx^2
(real).  Each request's initial state is made on the host when it arrives
and copied in by the server at admission; its final state is copied back
before the result is reported.  Latency = result time - submit time on the
server's clock.  Prints one JSON line; `--verify N` re-serves N sampled
requests alone afterwards and checks they give the same bits as in the mix.
The server detects ground-state requests whose start has no imaginary part
(the Gaussian starts here) and runs them on real storage, half the bytes
per point (GP_SERVER_REAL_AUTO; `--no-real-auto` turns that off).  With
`--real-states` the ground-state requests instead send their Gaussian as a
real array.
"""
from __future__ import annotations

import argparse
import json
import sys
import threading
import time

import numpy as np

from . import _binding as gp
from . import inputs

GRIDS = ((64, 64, 64), (96, 96, 96), (128, 128, 128), (160, 128, 96))
DX = 0.2


def schedule(rate: float, seconds: float, seed: int = 4, imag_fraction: float = 0.7) -> list:
    """Seeded arrivals: (time, kind, grid, trap, g) per request."""
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            return out
        kind = "imag" if rng.random() < imag_fraction else "real"
        grid = GRIDS[int(rng.integers(len(GRIDS)))]
        trap = tuple(float(v) for v in rng.uniform(0.5, 3.0, 3))
        g = float(rng.uniform(1.0, 500.0))
        out.append({"t": t, "kind": kind, "grid": grid, "trap": trap, "g": g})


def request_args(rq: dict, tol: float, imag_cap: int, real_steps: int) -> dict:
    imag = rq["kind"] == "imag"
    return {"dx": DX, "dt": (0.1 if imag else 0.005) * DX * DX, "trap": rq["trap"], "g": rq["g"],
            "mode": rq["kind"], "steps": imag_cap if imag else real_steps, "tol": tol if imag else 0.0}


def pct(v, q):
    return round(float(np.percentile(v, q)), 2) if len(v) else None


def run(rate=50.0, seconds=60.0, dtype="c64", budget_gib=2.0, slots=96, check_every=10, tol=1e-8,
        imag_cap=20000, real_steps=2000, verify=8, seed=4, real_states=False, graph=True, real_auto=True,
        log=None) -> dict:
    log = log or (lambda m: print(m, file=sys.stderr, flush=True))
    npd = np.complex128 if gp._dtype(dtype) == gp.C128 else np.complex64
    npr = np.float64 if npd is np.complex128 else np.float32

    def payload(rq):
        """The request's initial state: real storage for ground states when
        real_states (their Gaussian start is real)."""
        real = real_states and rq["kind"] == "imag"
        return inputs.separable_gaussian(rq["grid"], (DX,) * 3, rq["trap"], npr if real else npd)
    sched = schedule(rate, seconds, seed)
    keep = set(range(0, len(sched), max(1, len(sched) // max(verify, 1)))) if verify else set()
    keep = set(sorted(keep)[:verify])
    results, kept = {}, {}
    stop = threading.Event()

    with gp.Server(dtype=dtype, hbm_budget=int(budget_gib * (1 << 30)), max_slots=slots,
                   check_every=check_every, graph=graph, real_auto=real_auto) as srv:
        def collector():
            while not stop.is_set() or len(results) < len(sched):
                for r in srv.poll(wait=0.2):
                    if r["tag"] in keep:
                        kept[r["tag"]] = dict(r)
                    r["psi"] = None          # drop the host state of the others
                    results[r["tag"]] = r
                if stop.is_set() and len(results) >= len(sched):
                    return

        th = threading.Thread(target=collector, daemon=True)
        th.start()
        log(f"[serve] {len(sched)} requests over {seconds:.0f} s at {rate:g}/s, {dtype}, "
            f"budget {budget_gib:g} GiB, {slots} slots")
        t0 = time.perf_counter()
        next_log = t0 + 5.0
        late = []
        for i, rq in enumerate(sched):
            now = time.perf_counter()
            if now < t0 + rq["t"]:
                time.sleep(t0 + rq["t"] - now)
            late.append(time.perf_counter() - (t0 + rq["t"]))
            psi = payload(rq)
            srv.submit(psi, psi_out=psi, tag=i, **request_args(rq, tol, imag_cap, real_steps))
            if time.perf_counter() > next_log:
                st = srv.stats()
                log(f"[serve] t={time.perf_counter() - t0:5.1f}s submitted {i + 1} done {st['completed']} "
                    f"resident {st['resident']} queued {st['queued']}")
                next_log += 5.0
        while not srv.drain(5.0):
            st = srv.stats()
            log(f"[serve] draining: done {st['completed']} resident {st['resident']} queued {st['queued']}")
        stop.set()
        th.join()
        wall = time.perf_counter() - t0
        st = srv.stats()

        same = None
        if keep:
            same = 0
            for tag in sorted(keep):
                rq = sched[tag]
                psi = payload(rq)
                srv.submit(psi, psi_out=psi, tag=tag, **request_args(rq, tol, imag_cap, real_steps))
                alone = []
                while not alone:
                    alone = srv.poll(wait=1.0)
                a, m = alone[0], kept[tag]
                if a["status"] == m["status"] == 0 and a["steps"] == m["steps"] and \
                        np.array_equal(a["psi"], m["psi"]) and a["obs"]["mu"] == m["obs"]["mu"]:
                    same += 1
            log(f"[serve] {same}/{len(keep)} sampled requests give the same bits alone as in the mix")

    res = [results[i] for i in range(len(sched))]
    ok = [r for r in res if r["status"] == 0]
    lat = [1e3 * (r["t_done"] - r["t_submit"]) for r in ok]
    wait_ms = [1e3 * (r["t_admit"] - r["t_submit"]) for r in ok]
    by = {}
    for kind in ("imag", "real"):
        lk = [1e3 * (r["t_done"] - r["t_submit"]) for r, q in zip(res, sched) if q["kind"] == kind and r["status"] == 0]
        by[kind] = {"requests": sum(1 for q in sched if q["kind"] == kind), "p50_ms": pct(lk, 50),
                    "p99_ms": pct(lk, 99)}
    conv = [r["converged"] for r, q in zip(res, sched) if q["kind"] == "imag" and r["status"] == 0]
    span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
    pts = sum(r["steps"] * int(np.prod(q["grid"])) for r, q in zip(res, sched) if r["status"] == 0)
    return {
        "workload": f"serve-poisson-{rate:g}/s-{seconds:g}s", "dtype": dtype,
        "storage": ("complex128" if npd is np.complex128 else "complex64") +
                   (f"; ground states sent as real {np.dtype(npr).name}" if real_states else
                    (f"; ground states with real starts on {np.dtype(npr).name} (detected)" if real_auto else "")),
        "reductions": "f64", "requests": len(sched), "completed_ok": len(ok),
        "imag_converged": f"{sum(conv)}/{len(conv)}",
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "mean": round(float(np.mean(lat)), 2) if lat else None,
                       "max": round(max(lat), 2) if lat else None},
        "admission_wait_ms": {"p50": pct(wait_ms, 50), "p99": pct(wait_ms, 99)},
        "by_kind": by,
        "throughput_rps": round(len(ok) / span, 2), "offered_rps": rate,
        "pt_steps_per_s": pts / span, "makespan_s": round(span, 2), "wall_s": round(wall, 2),
        "submit_lateness_ms_p99": pct([1e3 * v for v in late], 99),
        "engine_seconds": {"copy_in": round(st["seconds_copy_in"], 2), "copy_out": round(st["seconds_copy_out"], 2),
                           "rounds": round(st["seconds_rounds"], 2)},
        "max_resident": st["max_resident"], "bytes_peak": st["bytes_peak"], "bytes_budget": st["bytes_budget"],
        "slots": slots, "check_every": check_every, "graph": graph, "rounds": st["quanta"],
        "graph_captures": st["graph_captures"],
        "same_alone_and_in_mix": None if same is None else f"{same}/{len(keep)}",
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--seconds", type=float, default=60.0)
    ap.add_argument("--dtype", default="c64", choices=["c64", "c64_f64", "c128"])
    ap.add_argument("--budget-gib", type=float, default=2.0)
    ap.add_argument("--slots", type=int, default=96)
    ap.add_argument("--check-every", type=int, default=10)
    ap.add_argument("--verify", type=int, default=8)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--real-states", action="store_true",
                    help="ground-state requests carry real states and run on real storage")
    ap.add_argument("--no-graph", action="store_true", help="launch the rounds' steps without graph replay")
    ap.add_argument("--no-real-auto", action="store_true",
                    help="keep real-start ground states on complex storage")
    a = ap.parse_args()
    out = run(a.rate, a.seconds, a.dtype, a.budget_gib, a.slots, a.check_every, verify=a.verify, seed=a.seed,
              real_states=a.real_states, graph=not a.no_graph, real_auto=not a.no_real_auto)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
