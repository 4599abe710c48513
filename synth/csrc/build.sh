#!/usr/bin/env bash
# Builds libsynth.so (GPU twin of the synthetic-input generator) for gfx950.
set -euo pipefail
here="$(cd "$(dirname "$0")" && pwd)"
hipcc --offload-arch=gfx950 -O3 -std=c++17 -fPIC -shared -ffp-contract=off \
  -Xclang -target-feature -Xclang -packed-fp32-ops \
  "$here/synth_gpu.hip" -o "$here/../libsynth.so"
