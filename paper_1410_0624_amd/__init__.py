"""colden: tree-based column densities (Valdivia & Hennebelle 2014) on
MI355X.  The column-density path lives in the HIP library libcolden.so
(C ABI in include/colden.h); `colden` is its Python binding and `synth` the
seeded input generators."""
