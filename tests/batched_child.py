"""Runs the batched problems of test_gpu_batched in a process of its own (the
hardware-queue count is fixed when the HIP runtime starts) and stores the
final factors and scores in an .npz file named on the command line."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402

from test_gpu_batched import SHAPES, _problem, _run_batched  # noqa: E402


def main(out: str) -> None:
    restarts = 3
    problems = [_problem(n, k, seed=100 + i, three=t, restarts=restarts) for i, (n, k, t) in enumerate(SHAPES)]
    _, run = _run_batched(problems, restarts)
    arrays = {}
    for i in range(len(problems)):
        arrays[f"phi{i}"] = run.Phi[i].cpu().numpy()
        arrays[f"score{i}"] = run.scores[i].cpu().numpy()
    np.savez(out, **arrays)
    print("child done", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
