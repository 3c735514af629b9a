"""RandomizedNNLS on MI355X: the randomized Hadamard sketch of [A | b] and the
Lawson-Hanson solve of the sketched problem, as hand-written HIP kernels for
gfx950 behind the C-ABI library ``librnnls.so``.

``paper_0812_4547_amd.rnnls`` is the Python binding (argument marshalling
only).  ``paper_0812_4547_amd.workloads`` draws the seeded synthetic inputs.
"""
__all__ = ["rnnls", "workloads"]
