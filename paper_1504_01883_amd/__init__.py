"""Depth-fused LBP face features and SVM scoring on MI355X (arXiv 1504.01883).

The compute path is the HIP library ``liblbpf.so`` (C ABI in include/lbpf.h);
``paper_1504_01883_amd.lbpf`` is its thin ctypes binding and
``paper_1504_01883_amd.synth`` draws the seeded synthetic inputs. Import the
submodules explicitly; this package file imports nothing, so the generator
works on machines without the built library.
"""
