# Address- and undefined-behaviour-sanitizer build of the CPU oracle, for
# the sanitized run of its pins (test infrastructure only; the library is
# loaded into a Python process started with libasan preloaded).
CC ?= gcc
SANFLAGS = -O2 -g -std=c11 -fopenmp -ffp-contract=off -fPIC -Wall -Wextra -D_DEFAULT_SOURCE \
           -fsanitize=address,undefined -fno-sanitize-recover=undefined -fno-omit-frame-pointer

liboracle_san.so: oracle.c oracle.h
	$(CC) $(SANFLAGS) -shared -o $@ oracle.c -lm
