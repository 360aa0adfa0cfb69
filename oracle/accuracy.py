"""Accuracy of the batch schedule against sequential SF_F -- TEST INFRASTRUCTURE ONLY.

Statistics over the CPU oracle's answers, for the measurement leg of the
benchmark and for the tests; the product path never imports this module.

For one workload (sketch shape, op stream, query keys) and one schedule batch
size b it runs the oracle twice -- strict sequential SF_F (Sections 3.4 and
3.5) and the deterministic batch schedule -- and reports:

* ARE and AAE of each mode against the exact net counts f over the queried
  keys with f > 0 (the paper's error metrics, Section 5.1; relative error is
  undefined at f = 0).  Slim counters saturate at 65535, so a key's error is
  taken against f' = min(f, 65535).
* ARE and AAE of batch against seq (|q_batch - q_seq| over the same keys).
* The certified per-key bound on that difference.  Both modes keep every
  answer inside [f', U(e)] with U(e) = min(65535, min_i max_k B_i[h_i(e)][k])
  (Appendix II gives the lower end, Appendix I the upper), and both reach the
  same Fat, so |q_batch - q_seq| <= U(e) - f'(e) for every key.  AAE_bound and
  ARE_bound are the means of that bound (absolute, and divided by f).
* The tolerance used to choose b: ARE_batch <= 1.10 * ARE_seq + 1e-3.

Running ``python -m oracle.accuracy`` prints the table of ARE against b for
the benchmark workloads (the "Choosing b" table of the design notes).
"""
from __future__ import annotations

import threading
import time

import numpy as np

from . import Sketch

SLIM_MAX = 65535
TOL_REL, TOL_ABS = 1.10, 1e-3


def _rows(a: np.ndarray) -> np.ndarray:
    return a if a.ndim == 1 else np.ascontiguousarray(a).view(np.dtype((np.void, a.shape[1]))).ravel()


def exact_counts(keys: np.ndarray, ops, queries: np.ndarray) -> np.ndarray:
    """Net count (inserts minus deletes) of every query key; 0 for keys never seen."""
    k, q = _rows(keys), _rows(queries)
    uniq, inv = np.unique(k, return_inverse=True)
    sign = np.ones(k.shape[0], np.int64) if ops is None else np.where(np.asarray(ops) == 1, -1, 1)
    cnt = np.bincount(inv.ravel(), weights=sign, minlength=uniq.shape[0]).astype(np.int64)
    pos = np.searchsorted(uniq, q)
    pos[pos >= uniq.shape[0]] = 0
    return np.where(uniq[pos] == q, cnt[pos], 0)


def errors(answers: np.ndarray, f: np.ndarray) -> dict:
    """ARE and AAE of answers against f' = min(f, 65535) over keys with f > 0."""
    m = f > 0
    if not m.any():
        return {"are": 0.0, "aae": 0.0, "keys": 0}
    a = answers.astype(np.int64)[m]
    fp = np.minimum(f[m], SLIM_MAX)
    err = np.abs(a - fp)
    return {"are": float(np.mean(err / f[m])), "aae": float(np.mean(err)), "keys": int(m.sum())}


def certified_bound(sk: Sketch, queries: np.ndarray, f: np.ndarray) -> dict:
    """Mean of U(e) - f'(e) (absolute and over f) for keys with f > 0, from the final
    Fat of sk, which is the same in every update mode."""
    fat = sk.fat()
    bmax = fat.max(axis=2).astype(np.int64)          # [d][w] bucket maxima
    h, _ = sk.indices(queries)
    u = np.min(np.stack([bmax[i][h[:, i]] for i in range(sk.d)]), axis=0)
    u = np.minimum(u, SLIM_MAX)
    m = f > 0
    if not m.any():
        return {"aae_bound": 0.0, "are_bound": 0.0}
    gap = u[m] - np.minimum(f[m], SLIM_MAX)
    return {"aae_bound": float(np.mean(gap)), "are_bound": float(np.mean(gap / f[m]))}


def run_modes(d, w, z, key_bytes, keys, ops, queries, b, seed_base=1, modes=("seq", "batch")):
    """Runs the requested oracle modes in parallel threads (the oracle call releases the
    interpreter lock).  Returns {mode: (sketch, answers, seconds)}."""
    out, errs = {}, []

    def one(mode):
        try:
            sk = Sketch(d, w, z, key_bytes, seed_base)
            t0 = time.perf_counter()
            rc = sk.seq(keys, ops) if mode == "seq" else sk.batch(keys, ops, b)
            if rc:
                raise RuntimeError(f"oracle {mode} failed: {rc}")
            el = time.perf_counter() - t0
            out[mode] = (sk, sk.query(queries), el)
        except Exception as e:  # surfaced below
            errs.append(e)

    th = [threading.Thread(target=one, args=(m,)) for m in modes]
    for t in th:
        t.start()
    for t in th:
        t.join()
    if errs:
        raise errs[0]
    return out


def report(d, w, z, key_bytes, keys, ops, queries, b, seed_base=1, batch_answers=None, runs=None) -> dict:
    """Accuracy block of one workload at schedule batch b.  batch_answers: the batch
    schedule's answers if already known (they are computed by the oracle otherwise)."""
    f = exact_counts(keys, ops, queries)
    if runs is None:
        modes = ("seq",) if batch_answers is not None else ("seq", "batch")
        runs = run_modes(d, w, z, key_bytes, keys, ops, queries, b, seed_base, modes)
    seq_sk, q_seq, t_seq = runs["seq"]
    q_b = batch_answers if batch_answers is not None else runs["batch"][1]
    e_seq, e_b = errors(q_seq, f), errors(q_b, f)
    m = f > 0
    diff = np.abs(q_b.astype(np.int64) - q_seq.astype(np.int64))[m]
    vs = {"are": float(np.mean(diff / f[m])) if m.any() else 0.0,
          "aae": float(np.mean(diff)) if m.any() else 0.0,
          "max_abs": int(diff.max()) if m.any() else 0,
          "keys_differing": int((diff > 0).sum())}
    bound = certified_bound(seq_sk, queries, f)
    absent = ~m & (f == 0)
    rep = {
        "b": int(b), "queried_keys_f_pos": int(m.sum()),
        "seq": {k: round(v, 6) if isinstance(v, float) else v for k, v in e_seq.items()},
        "batch": {k: round(v, 6) if isinstance(v, float) else v for k, v in e_b.items()},
        "batch_vs_seq": {k: round(v, 6) if isinstance(v, float) else v for k, v in vs.items()},
        "certified": {k: round(v, 6) for k, v in bound.items()},
        "within_certified": bool(vs["aae"] <= bound["aae_bound"] + 1e-12
                                 and vs["are"] <= bound["are_bound"] + 1e-12),
        "tolerance": f"ARE_batch <= {TOL_REL} x ARE_seq + {TOL_ABS}",
        "within_tolerance": bool(e_b["are"] <= TOL_REL * e_seq["are"] + TOL_ABS),
        "absent_keys": {"n": int(absent.sum()),
                        "mean_answer_batch": round(float(q_b[absent].mean()), 4) if absent.any() else 0.0,
                        "frac_nonzero_batch": round(float((q_b[absent] > 0).mean()), 6) if absent.any() else 0.0},
        "seq_oracle_s": round(t_seq, 2),
    }
    return rep


def _table():
    """ARE of sequential SF_F and of the batch schedule at several b, per workload."""
    import sfgen
    rows = []
    cases = [("32M ops, Zipf 0.6 (w = 2^20)", lambda: sfgen.config_main(0.6), [21, 22, 23, 24]),
             ("32M ops, Zipf 1.0 (w = 2^20)", lambda: sfgen.config_main(1.0), [21, 22, 23, 24]),
             ("32M ops, Zipf 1.4 (w = 2^20)", lambda: sfgen.config_main(1.4), [21, 22, 23, 24]),
             ("1M inserts, Zipf 1.0 (w = 2^14)", sfgen.config_small, [16, 18, 20]),
             ("128M flows, Zipf 1.2 (w = 2^21, d = 8)", sfgen.config_flows, [20, 21, 22, 23])]
    for name, gen, logs in cases:
        wl = gen()
        f = exact_counts(wl.keys, wl.ops, wl.queries)
        runs = run_modes(wl.d, wl.w, wl.z, wl.key_bytes, wl.keys, wl.ops, wl.queries, 1, modes=("seq",))
        a_seq = errors(runs["seq"][1], f)["are"]
        cells = [f"seq {a_seq:.5g}"]
        got = {}

        def one(lg):
            r = run_modes(wl.d, wl.w, wl.z, wl.key_bytes, wl.keys, wl.ops, wl.queries, 1 << lg,
                          modes=("batch",))
            got[lg] = errors(r["batch"][1], f)["are"]

        th = [threading.Thread(target=one, args=(lg,)) for lg in logs]
        for t in th:
            t.start()
        for t in th:
            t.join()
        for lg in logs:
            ok = got[lg] <= TOL_REL * a_seq + TOL_ABS
            cells.append(f"2^{lg}: {got[lg]:.5g}{'' if ok else ' (outside)'}")
        rows.append(f"| {name} | " + " | ".join(cells) + " |")
        print(rows[-1], flush=True)
    return rows


if __name__ == "__main__":
    _table()
