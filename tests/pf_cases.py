"""Inputs of the phase-field relaxation parity tests (shared by the GPU
tests and the CPU check that these inputs are well conditioned)."""
import workloads

# (grid n = (nx, ny, nz), spacings h, relaxation steps)
CASES = [((70, 13, 37), (0.25, 0.25, 0.25), 25),    # ragged x tiles and z chunk
         ((130, 21, 70), (0.25, 0.25, 0.25), 25),   # 3 tiles along every axis, ragged
         ((130, 9, 3), (0.2, 0.3, 0.25), 25),       # unequal spacings, thin y and z
         ((1, 1, 40), (1.0, 1.0, 0.2), 25),         # one node wide in x and y
         ((3, 2, 1), (0.25, 0.25, 0.25), 3)]        # smaller than the halo


def case_input(i):
    n, h, iters = CASES[i]
    return workloads.step_phase_field(n, h, seed=100 + i), h, iters
