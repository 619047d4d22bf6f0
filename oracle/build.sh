#!/bin/sh
# Builds the CPU oracle (test infrastructure).  Portable x86-64-v3 code so the library built here
# also runs on other hosts.
set -e
here="$(cd "$(dirname "$0")" && pwd)"
gcc -O2 -march=x86-64-v3 -fopenmp -fPIC -shared -Wall -Wno-unused-function \
    -o "$here/liboracle.so" "$here/bpm_oracle.c" -lm
