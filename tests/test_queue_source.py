"""The work-queue evolve kernel repeats the per-slot body of evolve_kernel
(it sits in its own translation unit so that the one-slot kernels' code is
unchanged, and so cannot call a shared function without changing them).
This keeps the two copies from drifting apart: the per-slot statements of
both kernels, comments and layout aside, must be the same."""
import os
import re

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2604_13144_amd", "csrc")


def per_slot_body(path, kernel):
    src = open(os.path.join(CSRC, path)).read()
    start = src.index(f"void {kernel}(")
    body = src[start:]
    a = body.index("const Slot S = make_slot<MIX>(a, slot, Jl);")
    b = body.index("store_state(a, slot, sh, layer0 + n_layers);", a)
    text = body[a:b + len("store_state(a, slot, sh, layer0 + n_layers);")]
    text = re.sub(r"//[^\n]*", "", text)
    return re.sub(r"\s+", " ", text).strip()


def test_queue_kernel_repeats_the_evolve_kernel_body():
    one = per_slot_body("kernels.hip", "evolve_kernel")
    queued = per_slot_body("queue.hip", "evolve_queue_kernel")
    assert len(one) > 500
    assert one == queued


def test_queue_translation_unit_leaves_out_the_kernels_file_launchers():
    src = open(os.path.join(CSRC, "kernels.hip")).read()
    # everything from the first kernel to the end of the launchers is guarded
    first_kernel = src.index("__global__")
    guard = src.rindex("#ifndef TEPAI_ENGINE_ONLY", 0, first_kernel)
    assert "__global__" not in src[:guard]
    assert src.count("#ifndef TEPAI_ENGINE_ONLY") == src.count("#endif  // TEPAI_ENGINE_ONLY") == 2
    q = open(os.path.join(CSRC, "queue.hip")).read()
    assert q.index("#define TEPAI_ENGINE_ONLY") < q.index('#include "kernels.hip"')
