// Continuous-batching solve server (not yet built).
