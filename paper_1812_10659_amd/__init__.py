"""LoLa-style encrypted inference (BFV over RNS) on MI355X: the HIP library
behind include/lola.h and its Python binding (paper_1812_10659_amd.lola)."""
