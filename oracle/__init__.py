"""Plain FP64 CPU oracle for RandomizedNNLS (Boutsidis & Drineas, "Random
Projections for the Nonnegative Least-Squares Problem").

TEST INFRASTRUCTURE ONLY.  This package is what the GPU library is checked
against.  Only the test-suite, the smoke check of ``__graft_entry__`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path
(``paper_0812_4547_amd``) never does, and shares no code with it: the two sides
only consume the same seeded inputs from ``paper_0812_4547_amd.workloads``.

Everything here is written for clarity, not speed: FP64 arithmetic, the
transforms and the active-set solver taken step by step in the paper's order.

Modules
-------
rng          counter-based random streams for the diagonal D and the row
             sample S of Algorithm 1 (the paper only fixes the probabilities;
             the concrete generator is this project's reading, restated from
             the published SplitMix64 finalizer).
hadamard     Walsh-Hadamard matrix in Sylvester (natural) order, its fast
             transform, and the sketch [H~ D A | H~ D b] of Algorithm 1.
nnls         Lawson-Hanson active-set NNLS (Definition 1), KKT certificate,
             brute force over supports, unconstrained least squares.
rand_nnls    Algorithm 1 end to end; its repetition over seeds; the box-bounded
             form of step 5.
bvls         least squares with box bounds lo <= x <= hi (bounded-variable
             active set), brute force over bound/free assignments.
nmf          alternating NNLS for a nonnegative factorisation.
diagnostics  realised subspace-embedding distortion (Lemma 1) and the
             row-norm flattening of Lemma 2, plus the proof chain of Theorem 1.
learned      per-column features, the passive-set perceptron (forward, loss,
             gradient, Adam step) of the learned warm start, in FP64.
"""
