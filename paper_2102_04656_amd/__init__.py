"""MI355X-native exact Hamming kNN-graph builder (Binary Distributed Graph, Sec. 3.2).

The compute path is the HIP library ``libbdg.so`` (C ABI, declared in
``include/bdg.h``); ``paper_2102_04656_amd.bdg`` is its thin ctypes binding.
Importing this package loads nothing; the binding loads the library on first use
and fails loudly if it is missing.
"""
__version__ = "0.1.0"
