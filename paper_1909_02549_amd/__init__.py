"""MI355X (gfx950) minibatched spiking-network hot path: HIP kernels behind a C ABI."""
