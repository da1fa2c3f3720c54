"""FP64 CPU oracle for the split-step two-component GPE -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may import this
package.  It shares no code with the HIP path; both sides only share the seeded workload
generators in ``workloads``.
"""
from .gpe import OracleGPE, exp2x2, apply2x2
from .observables import phase_separation, population_radius, winding

__all__ = ["OracleGPE", "exp2x2", "apply2x2", "phase_separation", "population_radius", "winding"]
