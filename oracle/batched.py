"""Many independent TR problems stepped one after another (CPU oracle;
test infrastructure only).  Each problem follows Algorithm TR-BRSGD exactly
as a single run would; batching changes no arithmetic."""
from __future__ import annotations

from . import brsgd


def run_all(problems, steps: int):
    """problems: list of (State, X, Config); advances each by ``steps``."""
    for state, X, cfg in problems:
        for _ in range(steps):
            brsgd.step(state, X, cfg)
    return problems
