"""MI355X (gfx950) directed-distance-field hot path: HIP kernels behind a C ABI.

The compiled library and its Python binding live in `ddf` (loaded lazily);
`inputs` holds the seeded synthetic workloads."""
