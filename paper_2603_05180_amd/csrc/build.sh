#!/usr/bin/env bash
# Builds libcrisp.so (the engine) for gfx950.  Usage: build.sh [out_dir]
set -euo pipefail
here="$(cd "$(dirname "$0")" && pwd)"
root="$(cd "$here/../.." && pwd)"
out="${1:-$here/..}"
hipcc --offload-arch=gfx950 -O3 -std=c++17 -fPIC -shared -ffp-contract=off \
  -Xclang -target-feature -Xclang -packed-fp32-ops \
  -I "$root/include" -I "$here" \
  "$here/crisp.hip" -o "$out/libcrisp.so"
