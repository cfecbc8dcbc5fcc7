#!/bin/bash
# Host-code sanitizer runs of the engine library (CPU only, no GPU needed):
#   thread   ThreadSanitizer on the server (prep, scheduler, batch runners,
#            copy threads) in its scheduler test mode
#   address  AddressSanitizer + UndefinedBehaviorSanitizer on the same
#            driver (request copies, basis builder and its validation)
# Device code is compiled as usual; only host code is instrumented.
# Usage: tests/sanitize/run.sh thread|address [outdir]
set -euo pipefail
KIND=${1:-thread}
ROOT=$(cd "$(dirname "$0")/../.." && pwd)
OUT=${2:-$ROOT/_build/sanitize_$KIND}
mkdir -p "$OUT"
case "$KIND" in
  thread)  SAN="-Xarch_host -fsanitize=thread" ; LSAN="-fsanitize=thread" ;;
  address) SAN="-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-sanitize-recover=undefined" ; LSAN="-fsanitize=address,undefined -fno-sanitize-recover=undefined" ;;
  *) echo "usage: $0 thread|address [outdir]"; exit 2 ;;
esac
HIPCC=${HIPCC:-/opt/rocm/bin/hipcc}
FLAGS="--offload-arch=gfx950 -O1 -g -std=c++17 -fPIC -Xclang -target-feature -Xclang -packed-fp32-ops -I$ROOT/include"
$HIPCC $FLAGS -shared $SAN "$ROOT"/paper_2512_18010_amd/csrc/*.hip "$ROOT"/paper_2512_18010_amd/csrc/*.cpp \
    -o "$OUT/libscarff_san.so" -lpthread
clang_host=/opt/rocm/lib/llvm/bin/clang++
$clang_host -O1 -g -std=c++17 $LSAN -I"$ROOT/include" "$ROOT/tests/sanitize/server_stress.cpp" \
    -L"$OUT" -Wl,-rpath,"$OUT" -lscarff_san -lpthread -o "$OUT/server_stress"
"$OUT/server_stress"
