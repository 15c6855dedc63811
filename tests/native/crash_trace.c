/*
 * Test-run diagnostics: on a fatal signal (SIGSEGV, SIGBUS, SIGILL, SIGFPE)
 * prints the faulting address and the native call stack to stderr (a frame
 * inside a local function of libpchase.so shows as object+offset, which
 * addr2line resolves against the same build); then
 * hands the signal back to the handler installed before it (Python's
 * faulthandler, which adds the Python stacks and ends the process).
 * Loaded by tests/conftest.py when built (__graft_entry__.build()).
 */
#define _GNU_SOURCE
#include <execinfo.h>
#include <signal.h>
#include <stdio.h>
#include <string.h>
#include <unistd.h>

static struct sigaction prev[65];

static void handler(int sig, siginfo_t *si, void *uc)
{
    (void)uc;
    char buf[512];
    int n = snprintf(buf, sizeof buf, "native stack (signal %d, address %p):\n", sig, si ? si->si_addr : NULL);
    if (n > 0) (void)!write(2, buf, (size_t)n);
    void *pcs[64];
    int k = backtrace(pcs, 64);
    backtrace_symbols_fd(pcs, k, 2);   /* object(+offset) or object(symbol+offset) per frame */
    /* the previous handler takes over: a fault re-executes the faulting
     * instruction on return and is delivered to it */
    sigaction(sig, &prev[sig], NULL);
}

__attribute__((constructor)) static void install(void)
{
    const int sigs[] = {SIGSEGV, SIGBUS, SIGILL, SIGFPE};
    for (unsigned i = 0; i < sizeof sigs / sizeof sigs[0]; ++i) {
        struct sigaction sa;
        memset(&sa, 0, sizeof sa);
        sa.sa_sigaction = handler;
        sa.sa_flags = SA_SIGINFO | SA_ONSTACK;
        sigemptyset(&sa.sa_mask);
        sigaction(sigs[i], &sa, &prev[sigs[i]]);
    }
}
