"""CPU FP64 oracle — test infrastructure only.

Plain, slow, readable NumPy code that states what the MI355X library must
compute: a plain tensor-train (TT) library, the paper's SDP encodings in TT
form, a dense primal-dual interior-point method for the same SDPs, the dense
Newton systems, and a reference TT interior-point method built from explicit
frame matrices.  Only the test-suite, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product library never does, and
nothing here imports the product library.
"""
