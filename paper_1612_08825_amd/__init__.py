"""MI355X (gfx950) direct n-D convolution and multi-scale time-to-contact.

The compute path is the HIP library ``libttcconv.so`` behind the C ABI in
``include/ttcconv.h``; ``paper_1612_08825_amd.api`` is its Python binding
(torch tensors in, device results out; import it explicitly, it loads torch)
and ``paper_1612_08825_amd.synth`` generates the seeded synthetic workloads.
"""
