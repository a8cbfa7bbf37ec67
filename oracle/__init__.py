"""FP64 oracle for VOctree rendering (NeuVV, arXiv 2202.06088).

TEST INFRASTRUCTURE ONLY. Nothing in the product package imports, links or
calls anything here; only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may. The oracle shares no code with the
GPU path: it has its own basis evaluation, its own traversal (a leaf-level
digital differential analyser over a hash set of occupied cells, not an
octree) and its own compositing, all in float64.

Modules
-------
hh       real 4-D hyperspherical harmonics from their definition (Sec. 4.1,
         Eq. 2-3; Appendix A.1-A.2), numpy.
core     ctypes front end of ``render.c`` (FP64 renderer, adjoint, pinhole
         rays) plus the depth-aware compositing of Alg. 1 in numpy.
"""
