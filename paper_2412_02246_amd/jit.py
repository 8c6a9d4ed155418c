"""Compiling many plans at once.  Run-time compilation is serialised inside one
process, so the contraction kernels of several plans are compiled in worker
processes (started with 'spawn'; they make no HIP device call) and installed in the
parent's plans with Plan.set_code.  Call it before the parent process first uses the
GPU."""
import multiprocessing
from concurrent.futures import ProcessPoolExecutor


def _compile_one(spec):
    from .plan import Plan
    n, edges, kw = spec
    return Plan(n, edges, **kw).code()


def compile_plans(plans, specs, workers=8):
    """plans[i] was built from specs[i] = (n, edges, kwargs); compile them all and install
    the code objects.  Plans that are already compiled are compiled again in workers
    only if asked for, so callers pass just the new ones."""
    if not plans:
        return plans
    if workers <= 1 or len(plans) == 1:
        for p in plans:
            p.compile()
        return plans
    ctx = multiprocessing.get_context("spawn")
    with ProcessPoolExecutor(max_workers=min(workers, len(plans)), mp_context=ctx) as ex:
        for p, (key, blob) in zip(plans, ex.map(_compile_one, specs)):
            p.set_code(key, blob)
    return plans
