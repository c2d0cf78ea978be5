"""Oracle potentials of the batched serving workload's problems at sampled
targets, computed in worker processes (spawned: they import only numpy and
the oracle, and rebuild each problem's inputs from its seeds)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_SAMPLE = 100


def sampled_reference(args):
    """(index, sampled target indices, oracle potentials (nvec, n_sample))."""
    i, spec = args
    import workloads
    from oracle import fmm
    pts = workloads.uniform_cube(spec["n"], spec["seed_points"])
    q = workloads.charges(spec["n"], spec["nvec"], spec["seed_charges"], "u01")
    s = workloads.sample_indices(spec["n"], N_SAMPLE, workloads.SEED_SAMPLES + 5 + i)
    ref = fmm.KiFMM(pts, pts, spec["depth"], spec["order"]).evaluate(q, s)
    return i, s, ref


THREAD_VARS = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")


def references(specs, workers=None):
    """One worker process per core, each single-threaded (the workers inherit
    the thread settings; numpy reads them when it is first imported)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    if workers is None:
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
    saved = {k: os.environ.get(k) for k in THREAD_VARS}
    for k in THREAD_VARS:
        os.environ[k] = "1"
    try:
        with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
            return sorted(ex.map(sampled_reference, list(enumerate(specs))), key=lambda r: r[0])
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
