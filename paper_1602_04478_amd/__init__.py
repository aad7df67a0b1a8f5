"""Colour-coding subgraph counting for treewidth-2 queries on MI355X (gfx950).

The computation lives in libcc.so (HIP kernels + C ABI, include/cc.h); this
package is its Python binding (``cc``) and build script (``build``)."""
