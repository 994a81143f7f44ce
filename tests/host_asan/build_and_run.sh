#!/bin/bash
# Builds the library's host code for the host only (no device code) with the
# address and undefined-behaviour sanitizers, links it with the emulated
# runtime and the driver, and runs the driver.  Usage: build_and_run.sh OUTDIR [ENGINE_SRC]
set -euo pipefail
HERE="$(cd "$(dirname "$0")" && pwd)"
ROOT="$(cd "$HERE/../.." && pwd)"
OUT="$1"
ENGINE="${2:-$ROOT/paper_1609_04104_amd/csrc/engine.hip}"
mkdir -p "$OUT"
HIPCC="${HIPCC:-/opt/rocm/bin/hipcc}"
SAN="-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-sanitize-recover=all"
COMMON="-x hip --offload-host-only -O1 -g -fno-omit-frame-pointer -std=c++17 -Wno-unused-result -Wno-unused-value -I$ROOT/include -I$ROOT/paper_1609_04104_amd/csrc"
"$HIPCC" $COMMON $SAN -c "$ENGINE" -o "$OUT/engine_host.o"
"$HIPCC" $COMMON $SAN -c "$HERE/hip_emul.cpp" -o "$OUT/hip_emul.o"
"$HIPCC" $COMMON $SAN -c "$HERE/engine_driver.cpp" -o "$OUT/engine_driver.o"
# link with the host compiler only: the emulation stands in for the HIP runtime
clang++ -fsanitize=address -fsanitize=undefined "$OUT/engine_host.o" "$OUT/hip_emul.o" "$OUT/engine_driver.o" \
    -o "$OUT/engine_driver" 2>/dev/null || \
    /opt/rocm/llvm/bin/clang++ -fsanitize=address -fsanitize=undefined "$OUT/engine_host.o" "$OUT/hip_emul.o" \
    "$OUT/engine_driver.o" -o "$OUT/engine_driver"
ASAN_OPTIONS=detect_leaks=0:abort_on_error=0 UBSAN_OPTIONS=print_stacktrace=1 "$OUT/engine_driver"
