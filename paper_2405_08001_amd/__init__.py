"""MI355X (gfx950) PNCG solver for the IPC incremental potential.

The compute path is libpncg.so (hand-written HIP); this package only binds
it.  ``Context`` wraps one library context; its methods carry the C ABI names
(``pncg_set_mesh``, ``pncg_step``, ...); ``Batch`` wraps the batched
entry points; ``simulate`` / ``Simulation`` (module ``autograd``) make a
rollout differentiable through the adjoint entry point.  The binding is loaded on first use
of any of its names and raises ImportError if the library has not been built
(``python -m paper_2405_08001_amd.build``); the build module itself does not
need the library.
"""
import importlib

_BINDING_NAMES = {
    "Context", "Batch", "PncgError", "pncg_create", "FP64", "MIXED", "TERM_DELTA_E", "TERM_GRAD_REL", "TERM_GRAD_ABS",
    "BARRIER_FULL", "ALPHA_INF_COMPONENT", "BETA_DK", "BETA_FR", "BETA_PRP", "BETA_CD", "BETA_HZ", "BETA_RULES", "SPLIT_OBJECTS", "MODEL_NH", "MODEL_SNH", "MODEL_ARAP", "MODEL_FCR", "MODELS", "CONTACT_SELF", "CONTACT_REST_EXCLUDE", "KIND_PT", "KIND_EE",
    "KIND_PG", "W_MAXITER", "E_INVAL", "E_STATE", "E_INVERTED", "E_NONFINITE", "E_PENETRATION", "E_HIP",
    "E_CAPACITY", "E_INDEFINITE", "EXPORTS", "LIB_PATH", "PROF_KINDS", "SCATTER_AUTO", "SCATTER_ATOMIC",
    "SCATTER_SEGMENTED", "NOALLOC_ITER_MAX", "E_CAPACITY",
}


_AUTOGRAD_NAMES = {"Simulation", "simulate"}


def __getattr__(name):
    if name in _BINDING_NAMES:
        mod = importlib.import_module("._lib", __name__)
        return getattr(mod, name)
    if name in _AUTOGRAD_NAMES:
        mod = importlib.import_module(".autograd", __name__)
        return getattr(mod, name)
    raise AttributeError(name)
