"""The boundary allocates device memory only in vmc_init.

Stepping calls (local energy, CTMC moves, gradient, estimator, AMSGrad,
batches) must allocate nothing, so that they can be captured in a hipGraph
and run in loops that may not allocate.  Without a GPU this is checked on the
source: every allocating or freeing HIP runtime call of the library sits in a
function that only vmc_init (allocation) or the handle's destruction (free)
reaches.
"""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1807_10633_amd", "csrc", "vmc.hip")

ALLOC = re.compile(r"\bhip(Malloc|MallocManaged|HostMalloc|ExtMallocWithFlags|MallocAsync|Free|FreeAsync|HostFree)\s*\(")


def _functions(src):
    """(name, body) of every top-level function definition, by brace matching."""
    out = []
    head = re.compile(r"^[A-Za-z_][\w:<>,\s\*&]*?\b([A-Za-z_]\w*)\s*\([^;{]*\)\s*(?:const\s*)?\{", re.M)
    for m in head.finditer(src):
        depth, i = 0, m.end() - 1
        while i < len(src):
            if src[i] == "{":
                depth += 1
            elif src[i] == "}":
                depth -= 1
                if depth == 0:
                    break
            i += 1
        out.append((m.group(1), src[m.start():i + 1]))
    return out


def test_allocation_only_at_init_and_free_only_at_destruction():
    src = open(SRC).read()
    funcs = _functions(src)
    allocating = {name for name, body in funcs if re.search(r"\bhip(Malloc|HostMalloc|ExtMallocWithFlags)\w*\s*\(", body)}
    freeing = {name for name, body in funcs if re.search(r"\bhip(Free|HostFree|FreeAsync)\s*\(", body)}
    # the table upload helper allocates, vmc_init allocates the parameter
    # copies, vmc_cps_init (a setup call) the correlator tables
    assert allocating <= {"upload", "vmc_init", "vmc_cps_init"}, allocating
    assert freeing <= {"free_ctx"}, freeing
    callers = {name for name, body in funcs if re.search(r"\bupload\s*\(", body) and name != "upload"}
    assert callers <= {"vmc_init", "vmc_cps_init"}, callers
    free_callers = {name for name, body in funcs if re.search(r"\bfree_ctx\s*\(", body) and name != "free_ctx"}
    assert free_callers <= {"vmc_init", "vmc_destroy"}, free_callers


def test_stepping_entry_points_reach_no_allocation():
    src = open(SRC).read()
    funcs = dict(_functions(src))
    for ep in ("vmc_local_energy", "vmc_ctmc_step", "vmc_ctmc_step_dev", "vmc_logderiv", "vmc_estimate",
               "vmc_amsgrad", "vmc_walkers_init", "vmc_walkers_refresh", "vmc_batch_local_energy",
               "vmc_batch_ctmc_step", "vmc_set_params", "vmc_set_cps", "vmc_ctmc_step_static", "vmc_logderiv_accumulate",
               "vmc_snapshot_weights", "vmc_gradient_combine"):
        assert ep in funcs, ep
        assert not ALLOC.search(funcs[ep]), ep
    # the helpers they launch through
    for helper in ("launch_sweep", "launch_refresh", "launch_batch", "launch_prec", "launch_one", "launch_hbm",
                   "launch_streams", "logderiv_contract"):
        if helper in funcs:
            assert not ALLOC.search(funcs[helper]), helper
