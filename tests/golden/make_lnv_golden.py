"""Write the stored oracle values of full Hotelling + LNV solves.

Calls only the FP64 CPU oracle (`oracle`) and the seeded input generator
(`synth`); nothing here touches the HIP library.  The GPU tests compare the
library's solve of the same seeded system with these values.

Cases:
  si4096_b9      4096-atom diamond Si (8x8x8 cells), 9 orbitals per atom,
                 S/H on 6 A, S^-1 on 8 A, L on 10 A: Hotelling to its floor,
                 then LNV to |dE| < 1e-8 Ha (hours on a few CPU cores, ~30 GB).
  si512_b9_disp  512 atoms (4x4x4 cells), Gaussian displacements sigma 0.05 A,
                 the same cutoffs: the L, S^-1 and S patterns are genuinely
                 sparse (191, 99 and 47 of 512 columns on the ideal lattice).

Stored per case (JSON): the Hotelling residual after every update, the
Gershgorin scale and the update count; the initial-guess traces; per LNV
iteration E, N, mu, alpha, beta, dE and Omega; the idempotency error of the
converged L; 64 seeded sample blocks of the
final S^-1 and L with their (row, column); the Frobenius norm of every block
row of both; wall times and the thread count of this run.

Usage:  python tests/golden/make_lnv_golden.py [--checkpoint DIR] si512_b9_disp [si4096_b9 ...]

With --checkpoint DIR the state after Hotelling and after every LNV iteration
is saved there (raw arrays), and so is every block product of the stage in
progress (the state restore and each LNV iteration) as it completes: a rerun
resumes from the last saved state and loads the saved products of the
interrupted stage in call order instead of recomputing them.  The oracle is
deterministic, so the resumed run computes the same bits as an uninterrupted
one; the stored stage times add each loaded product's original compute time to
the rerun's own.
"""
import json
import math
import os
import platform
import shutil
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O   # noqa: E402
import synth         # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

HOT_MAX_ITER, HOT_TOL = 100, 1e-12
TOL_E, MAX_LNV = 1e-8, 300
SAMPLES = 64


def case_system(name):
    if name == "si4096_b9":
        return synth.si4096_b9()
    if name == "si512_b9_disp":
        return synth.make_system("si512_b9_disp", 4, 9, synth.BIG_CUTOFFS, 7, displacement_sigma=0.05)
    raise ValueError(name)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def sample_blocks(M, rng):
    P = M.pattern
    slots = np.sort(rng.choice(P.nnz, size=min(SAMPLES, P.nnz), replace=False))
    rows = P.rows()[slots]
    return {"rows": rows.tolist(), "cols": P.cols[slots].tolist(),
            "blocks": [[float(v) for v in M.blocks[s].ravel()] for s in slots]}


def row_norms(M):
    P = M.pattern
    sq = np.einsum("nab,nab->n", M.blocks, M.blocks)
    per_row = np.add.reduceat(sq, P.rowptr[:-1]) if P.nnz else np.zeros(P.natoms)
    return [float(math.sqrt(v)) for v in per_row]


def log(*a):
    print(*a, flush=True)


def _save(ck, name, arr):
    np.save(os.path.join(ck, name + ".tmp.npy"), arr)
    os.replace(os.path.join(ck, name + ".tmp.npy"), os.path.join(ck, name + ".npy"))


def _load(ck, name):
    path = os.path.join(ck, name + ".npy")
    return np.load(path) if os.path.exists(path) else None


class ProductCache:
    """Stands in for the oracle's `product` while a checkpointed stage runs: the
    n-th product of the stage is saved on completion and, in a rerun of the same
    stage, loaded instead of recomputed."""

    def __init__(self, compute):
        self.compute = compute
        self.dir = None
        self.n = 0
        self.saved_s = 0.0      # original compute time of the products loaded
        self.load_s = 0.0       # time spent loading them
        self.save_s = 0.0       # time spent writing the computed ones

    def stage(self, path):
        self.dir, self.n, self.saved_s, self.load_s, self.save_s = path, 0, 0.0, 0.0, 0.0
        if path:
            os.makedirs(path, exist_ok=True)

    def drop(self, path):
        if path and os.path.isdir(path):
            shutil.rmtree(path)

    def __call__(self, A, B, pattern, prec=O.F64):
        if not self.dir:
            return self.compute(A, B, pattern, prec)
        base = os.path.join(self.dir, f"p{self.n:03d}")
        self.n += 1
        if os.path.exists(base + ".json"):
            t0 = time.perf_counter()
            with open(base + ".json") as f:
                m = json.load(f)
            C = O.Matrix(pattern, A.b, np.load(base + ".npy"))
            assert C.pattern.nnz == m["nnz"] and m["prec"] == prec
            self.load_s += time.perf_counter() - t0
            self.saved_s += m["s"]
            return C
        t0 = time.perf_counter()
        C = self.compute(A, B, pattern, prec)
        dt = time.perf_counter() - t0
        np.save(base + ".tmp.npy", C.blocks)
        os.replace(base + ".tmp.npy", base + ".npy")
        with open(base + ".tmp.json", "w") as f:
            json.dump({"s": dt, "nnz": int(pattern.nnz), "prec": prec}, f)
        os.replace(base + ".tmp.json", base + ".json")
        self.save_s += time.perf_counter() - t0 - dt
        return C

    def credit(self):
        """Seconds the loaded products took when computed, less the time spent loading them
        and saving the others: what the stage would have taken without checkpoints."""
        return self.saved_s - self.load_s - self.save_s


def run(name, ckdir=None):
    ck = None
    if ckdir:
        ck = os.path.join(ckdir, name)
        os.makedirs(ck, exist_ok=True)
    s = case_system(name)
    cut = s.cutoffs
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count())
    log(f"[{name}] {s.natoms} atoms, b={s.b}, cutoffs {cut}, {threads} threads")
    t_all = time.perf_counter()
    PS = O.create_pattern(s.positions, s.box, cut["S"])
    PZ = O.create_pattern(s.positions, s.box, cut["Z"])
    PL = O.create_pattern(s.positions, s.box, cut["L"])
    S = O.from_blocks(PS, s.b, s.S.rows, s.S.cols, s.S.blocks)
    H = O.from_blocks(PS, s.b, s.H.rows, s.H.cols, s.H.blocks)

    t0 = time.perf_counter()
    meta = json.load(open(os.path.join(ck, "meta.json"))) if ck and os.path.exists(os.path.join(ck, "meta.json")) \
        else None
    if meta is not None:
        hr = O.HotellingResult(O.Matrix(PZ, s.b, _load(ck, "Z")), meta["hot_status"], meta["hot_iterations"],
                               meta["hot_residuals"], meta["hot_alpha"])
        hot_s = meta["hot_s"]
        log(f"[{name}] Hotelling and {len(meta['iters'])} LNV iterations restored from {ck}")
    else:
        hr = O.hotelling_inverse(S, PZ, max_iter=HOT_MAX_ITER, tol=HOT_TOL)
        hot_s = time.perf_counter() - t0
    log(f"[{name}] Hotelling: status {hr.status}, {hr.iterations} updates, residuals "
        f"{hr.residuals[0]:.6e} -> {hr.residuals[-1]:.6e}, {hot_s:.1f} s")
    if hr.status != O.OK:
        raise RuntimeError(f"Hotelling failed with status {hr.status}")

    cache = ProductCache(O.product)
    if ck:
        O.product = cache
    t0 = time.perf_counter()
    if meta is not None and meta["iters"]:
        cache.stage(os.path.join(ck, f"restore{len(meta['iters'])}"))
        st = O.lnv_init(S, H, hr.Z, PL, s.n_electrons, tol_E=TOL_E, L0=O.Matrix(PL, s.b, _load(ck, "L")))
        cache.stage(None)
        st.n, st.E_prev, st.mu = meta["n"], meta["E_prev"], meta["mu"]
        st.D_prev, st.g_prev, st.Mg_prev = (O.Matrix(PL, s.b, _load(ck, k)) for k in ("D", "g", "Mg"))
        init_s = meta["init_s"]
    else:
        st = O.lnv_init(S, H, hr.Z, PL, s.n_electrons, tol_E=TOL_E)
        init_s = time.perf_counter() - t0
    log(f"[{name}] initial L: {init_s:.1f} s")
    iters, step_s = (list(meta["iters"]), list(meta["step_s"])) if meta is not None else ([], [])

    def checkpoint():
        if not ck:
            return
        if st.D_prev is not None:
            for k, M in (("L", st.L), ("D", st.D_prev), ("g", st.g_prev), ("Mg", st.Mg_prev)):
                _save(ck, k, M.blocks)
        else:
            _save(ck, "Z", hr.Z.blocks)
        m = {"hot_status": hr.status, "hot_iterations": hr.iterations, "hot_residuals": hr.residuals,
             "hot_alpha": hr.alpha, "hot_s": hot_s, "init_s": init_s, "n": st.n, "E_prev": st.E_prev,
             "mu": st.mu, "iters": iters, "step_s": step_s}
        with open(os.path.join(ck, "meta.tmp.json"), "w") as f:
            json.dump(m, f)
        os.replace(os.path.join(ck, "meta.tmp.json"), os.path.join(ck, "meta.json"))

    if meta is None:
        checkpoint()
    converged = bool(iters) and abs(iters[-1]["dE"]) < TOL_E and len(iters) > 1
    for it in range(len(iters) + 1, MAX_LNV + 1):
        if converged:
            break
        step_dir = os.path.join(ck, f"step{it}") if ck else None
        cache.stage(step_dir)
        t0 = time.perf_counter()
        r = O.lnv_step(st)
        step_s.append(time.perf_counter() - t0 + cache.credit())
        cache.stage(None)
        if r.status != O.OK:
            raise RuntimeError(f"LNV step {it} failed with status {r.status}")
        iters.append({"E": r.E, "N": r.N, "mu": r.mu, "alpha": r.alpha, "beta": r.beta,
                      "dE": r.dE, "Omega": r.Omega})
        log(f"[{name}] LNV {it:3d}  E={r.E:.12f}  dE={r.dE:+.3e}  N={r.N:.10f}  mu={r.mu:+.6e}  "
            f"alpha={r.alpha:.6e}  {step_s[-1]:.1f} s")
        checkpoint()
        if ck:
            cache.drop(step_dir)
            cache.drop(os.path.join(ck, f"restore{it - 1}"))
        if r.converged:
            converged = True
            break
    lnv_s = sum(step_s)
    cache.stage(os.path.join(ck, "final") if ck else None)
    e_idem = O.idempotency_error(st)
    cache.stage(None)
    log(f"[{name}] idempotency error of the converged L: {e_idem:.6e}")
    rng = np.random.default_rng(2205)
    out = {
        "case": name,
        "generator": {"ncell": [int(round(v / synth.A_SI)) for v in s.box], "b": s.b, "cutoffs_A": cut,
                      "seed": s.seed, "natoms": s.natoms, "n_electrons": s.n_electrons},
        "hotelling": {"max_iter": HOT_MAX_ITER, "tol": HOT_TOL, "status": hr.status,
                      "iterations": hr.iterations, "alpha": hr.alpha, "residuals": hr.residuals},
        "lnv": {"tol_E": TOL_E, "max_iter": MAX_LNV, "converged": converged, "iterations": iters,
                "E_final": iters[-1]["E"], "idempotency_error": e_idem},
        "Z_samples": sample_blocks(st.Z, rng),
        "L_samples": sample_blocks(st.L, rng),
        "Z_row_norms": row_norms(st.Z),
        "L_row_norms": row_norms(st.L),
        "L_norm": float(np.linalg.norm(st.L.blocks.ravel())),
        "timing": {"threads": threads, "cpu": cpu_model(), "hotelling_s": hot_s, "init_s": init_s,
                   "lnv_s": lnv_s, "lnv_step_s": step_s, "solve_s": hot_s + init_s + lnv_s,
                   "total_s": time.perf_counter() - t_all},
    }
    path = os.path.join(HERE, f"lnv_{name}.json")
    with open(path + ".tmp", "w") as f:
        json.dump(out, f, indent=0)
    os.replace(path + ".tmp", path)
    log(f"[{name}] wrote {path}: {len(iters)} LNV iterations, E = {iters[-1]['E']:.12f}, "
        f"solve {hot_s + init_s + lnv_s:.1f} s")


if __name__ == "__main__":
    args = sys.argv[1:]
    ckdir = None
    if args[:1] == ["--checkpoint"]:
        ckdir, args = args[1], args[2:]
    for name in args or ["si512_b9_disp"]:
        run(name, ckdir)
