"""MI355X-native construction of stable locally consistent grammars (LCG).

The package holds the ctypes binding of the HIP library ``liblcg.so``
(``lcg``), the seeded synthetic input generator (``datagen``), canonical
renaming for comparisons (``canon``) and the serving loop (``serve``).
"""
