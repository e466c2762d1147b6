"""MI355X (gfx950) betweenness centrality over a source set.

Brandes BC (paper: StarPlat, arXiv 2305.03317, Appendix Fig. "BC computation
in StarPlat") behind the C ABI of ``include/sp.h``:

* ``sp``      - ctypes binding of ``libsp.so`` (HIP kernels for gfx950),
* ``graphs``  - seeded synthetic CSR graphs (uniform, RMAT, road-like),
* ``_build``  - in-tree compilation of both native libraries.

Submodules are imported on use; nothing here touches the GPU at import.
"""
__all__ = ["sp", "graphs"]
