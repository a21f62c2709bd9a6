"""CPU oracle for the accelerated-SLM per-node split search (TEST INFRASTRUCTURE).

A plain, slow, FP64 NumPy statement of what the split search computes, written
from the paper (Fu et al., "Acceleration of Subspace Learning Machine via
Particle Swarm Optimization and Parallel Processing", arXiv 2208.07023):

* projection of samples onto unit directions (Sec. II-A, Eqs. (1)-(2));
* the threshold bipartition (Sec. II-A, Eqs. (3)-(4)) and the loss of the best
  threshold of each projected 1-D feature (Sec. III-B), under the Gini,
  entropy or MSE criterion;
* the particle swarm update and loop (Sec. III-A, Eqs. (11)-(12), Alg. 1) and
  its adaptive variant (oracle.apso; Sec. III-B);
* the binary tree built on the global-best split (Sec. III-B, Alg. 2);
* bfloat16 screening of a swarm evaluation with float32 re-scoring of the
  best few particles (oracle.screen);
* the discriminant feature test of a node and the swarm start in its top n
  channels (oracle.dft; Alg. 2);
* the original SLM's probabilistic search over the DFT-ranked channels
  (oracle.probsearch; Sec. II-B);
* bagged (forest) and boosted ensembles of SLM trees (oracle.ensemble; Sec. V).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the GPU path and imports nothing
from it; both sides take inputs from the seeded generators only.
"""
from . import philox, split, pso, apso, screen, dft, probsearch, tree, brute, ensemble  # noqa: F401
