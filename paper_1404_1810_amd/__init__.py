"""amqft: batched power-of-two complex DFT by the AM-QFT recursion
(Pasquini, arXiv:1404.1810), hand-written HIP kernels for AMD MI355X (gfx950)
behind a C ABI (include/amqft.h).

The torch-facing functions are imported lazily so that the input generators
(``paper_1404_1810_amd.inputs``) and the build script work without a GPU.
"""

__all__ = ["fft", "adjoint", "ifft", "amqft", "power_loss", "Plan", "ManyPlan", "exec_graph", "AMQFTFunction", "build"]


def __getattr__(name):
    if name in ("fft", "adjoint", "ifft", "amqft", "power_loss", "Plan", "AMQFTFunction", "get_plan", "ManyPlan",
                "exec_graph"):
        from . import api
        return getattr(api, name)
    if name == "build":
        from .build import build
        return build
    raise AttributeError(name)
