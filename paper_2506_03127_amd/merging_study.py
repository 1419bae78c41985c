"""Pre-merging against post-merging with the same MACGIC mask (Sec. 2.1 and
Sec. 3.1): how far the populations of the two orders part, and what each
stores, over the filter threshold theta.

Post-merging (the original scheme) extends every group by every pair and then
merges the children on the mask m; pre-merging merges the stored paths on the
reduced mask {m[i] - 1} first, so the expansion starts from fewer groups.  Here
neither order writes the children to memory (they merge on chip), so the
memory of a run is its stored groups; the study reports their peak and mean,
the path-steps, and the largest difference of the populations rho_ii(t).

    python -m paper_2506_03127_amd.merging_study        (needs the GPU)
"""
from __future__ import annotations

import time

import numpy as np

from . import quapi, workloads

RECORD_BYTES = 32


def run(wl, mode: int, theta: float, n_steps: int):
    b = wl.bath
    eta = quapi.quapi_eta(b.ohmic_alpha, b.ohmic_wc, [x for pk in b.peaks for x in pk], wl.beta, wl.dt, wl.K)
    g = quapi.Propagator(wl.H, wl.q, wl.dt, wl.K, eta, wl.rho0, mask=wl.mask, theta=theta, mode=mode,
                         max_steps=n_steps)
    t0 = time.perf_counter()
    g.step(n_steps)
    g.sync()
    el = time.perf_counter() - t0
    rho = g.rho_history(0, n_steps + 1)
    st = g.stats(1, n_steps)
    g.close()
    stored = np.array([s["n_stored"] for s in st], dtype=np.float64)
    return {"rho": rho, "stored_max": float(stored.max()), "stored_mean": float(stored.mean()),
            "path_steps": float(sum(s["n_children"] for s in st)), "seconds": el}


def compare(wl, thetas, n_steps: int):
    rows = []
    for th in thetas:
        pre = run(wl, quapi.QUAPI_PRE, th, n_steps)
        post = run(wl, quapi.QUAPI_POST, th, n_steps)
        M = wl.M
        pop = np.abs(np.real(np.einsum("tii->ti", pre["rho"]) - np.einsum("tii->ti", post["rho"]))).max()
        rows.append({"workload": wl.name, "M": M, "K": wl.K, "mask": wl.mask, "theta": th, "steps": n_steps,
                     "max_population_difference": float(pop),
                     "pre_stored_max": pre["stored_max"], "post_stored_max": post["stored_max"],
                     "stored_ratio_post_pre": post["stored_max"] / pre["stored_max"],
                     "pre_mean": pre["stored_mean"], "post_mean": post["stored_mean"],
                     "pre_path_steps": pre["path_steps"], "post_path_steps": post["path_steps"],
                     "pre_MB": pre["stored_max"] * RECORD_BYTES / 1e6, "post_MB": post["stored_max"] * RECORD_BYTES / 1e6,
                     "pre_s": pre["seconds"], "post_s": post["seconds"]})
    return rows


def table(rows) -> str:
    head = ("| system | theta | max pop. diff | stored groups pre / post (peak) | ratio post/pre | "
            "path-steps pre / post | store MB pre / post | s pre / post |")
    out = [head, "|" + "---|" * 8]
    for r in rows:
        out.append(f"| {r['workload']} | {r['theta']:.0e} | {r['max_population_difference']:.2e} | "
                   f"{r['pre_stored_max']:.3g} / {r['post_stored_max']:.3g} | {r['stored_ratio_post_pre']:.2f} | "
                   f"{r['pre_path_steps']:.3g} / {r['post_path_steps']:.3g} | {r['pre_MB']:.3g} / {r['post_MB']:.3g} | "
                   f"{r['pre_s']:.3f} / {r['post_s']:.3f} |")
    return "\n".join(out)


def main():
    rows = []
    rows += compare(workloads.structured_bath(), [1e-6, 1e-8, 1e-10, 1e-12], 1000)
    rows += compare(workloads.three_level(K=10, n_exact=6), [1e-6, 1e-8, 1e-10], 300)
    print(table(rows), flush=True)


if __name__ == "__main__":
    main()
