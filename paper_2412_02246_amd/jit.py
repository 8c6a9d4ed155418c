"""Compiling contraction code in parallel.  Run-time compilation is serialised inside
one process, so the parts of one or many plans are compiled in worker processes
(started with 'spawn'; they make no HIP device call) and installed in the parent's
plans with Plan.set_code.  Call it before the parent process first uses the GPU."""
import multiprocessing
from concurrent.futures import ProcessPoolExecutor


def _compile_part(task):
    from .plan import Plan
    (n, edges, kw), part = task
    return Plan(n, edges, **kw).code(part)


def compile_parts(plans, specs, workers=8):
    """plans[i] was built from specs[i] = (n, edges, kwargs); compile every part of every
    plan and install the code objects."""
    if not plans:
        return plans
    tasks = [(i, k) for i, p in enumerate(plans) for k in range(p.jit_parts)]
    if workers <= 1 or len(tasks) == 1:
        for p in plans:
            p.compile()
        return plans
    ctx = multiprocessing.get_context("spawn")
    with ProcessPoolExecutor(max_workers=min(workers, len(tasks)), mp_context=ctx) as ex:
        results = ex.map(_compile_part, [(specs[i], k) for i, k in tasks])
        for (i, k), (key, blob) in zip(tasks, results):
            plans[i].set_code(k, key, blob)
    return plans

