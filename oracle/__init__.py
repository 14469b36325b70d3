"""PEPSI reference oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, textbook CPU implementation of what the GPU path computes
(the server side of PEPSI PSI-cardinality, arXiv 2310.14565), used to check
the GPU library bit for bit.  Only the tests, the smoke entry point and the
CPU-baseline leg of the benchmark may import it; the GPU library never does,
and the two share no code.

Modules: params (scheme/protocol parameters), hashing (cuckoo and simple
hashing), cw (constant-weight codes), core (ctypes binding of the C core in
csrc/: negacyclic products, textbook FV, server computation), protocol
(client/server preparation and result extraction).
"""
