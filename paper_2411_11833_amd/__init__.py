"""MI355X-native particle cost / gradient / Adam step of differentiable
GPU-parallelized task and motion planning (cuTAMP, Shen et al.).

The package is deliberately light at import time: ``inputs`` (seeded synthetic
robots, scenes and skeletons) has no dependency on the compiled library, and
``binding`` / ``planner`` load ``libcutamp.so`` only when imported.
"""

__all__ = ["inputs", "binding", "planner"]
