"""MI355X-native data-driven BFS/SSSP hot path (IrGL worklist ForAll, nested
edge parallelism, cooperative worklist pushes, iteration-outlined persistent
loop with a grid-wide barrier).

Importing the package loads nothing native; the HIP library is loaded by
``paper_1607_05707_amd.irgl`` on first import and that import fails loudly
when the library has not been built.
"""
__version__ = "0.1.0"
